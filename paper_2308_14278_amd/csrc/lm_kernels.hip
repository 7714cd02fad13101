// lm_kernels.hip -- gfx950 kernels of liblensmap besides the shooting kernels
// (lm_device.h, instantiated per scheme and precision in lm_shoot_inst.hip),
// and the entry points that launch every kernel.
//
//  k_coeffs       far-field Taylor coefficients of every level-2 cell (Sec. 3.2.2):
//                 a_n = -sum_{far k} m_k / (z_k - z_c)^(n+1); lens tiles staged
//                 in LDS, FP64 arithmetic (FP64 FMA issues at the unpacked
//                 FP32 rate on gfx950).
//  k_l1_expand    hierarchical far field (optional): series per level-1 cell,
//  k_l1_shift     re-expanded about every level-2 centre.
//  k_ptab         the column-offset table of the shooting kernels.
//  k_sum_u64, k_fill_u64   reductions and fills of count buffers.
//
// The shooting kernels (k_shoot_map: one workgroup per tile of level-2 cells;
// k_shoot_batch: persistent, tiles of many maps from a queue) sum the near
// lenses directly (Eq. 9) on offsets rebased to the cell centre (FP32, or FP64
// in the FP64 near-sum mode), add the far-field Taylor series and the macro
// map with the sheet term (Eq. 6) re-expanded per ray row, bin in FP64 pixel
// coordinates, and count (Sec. 3.2.3) through per-lane runs, a wave merge and
// an LDS window flushed to the uint64 map.
#include "lm_device.h"

namespace {

// A lens as staged for the coefficient sums: position, mass, level-1 cell.
template <class T>
struct alignas(16) CoefLens {
    T x, y, m;
    int I, J;
};

// Far-field coefficients: one level-2 cell per thread, lens tiles in LDS.
template <int PREC, int P>
__global__ __launch_bounds__(kWG) void k_coeffs(LmDesc d, int64_t ci0, int64_t cj0, int64_t nci,
                                                int64_t ncj, LmCoef* __restrict__ out)
{
    typedef typename std::conditional<PREC != 1, double, float>::type T;
    __shared__ CoefLens<T> sl[kWG];
    const int tid = threadIdx.x;
    const int64_t c = (int64_t)blockIdx.x * kWG + tid;
    const bool valid = c < nci * ncj;
    const int64_t ci = ci0 + (valid ? c % nci : 0), cj = cj0 + (valid ? c / nci : 0);
    const int I = (int)(ci / d.Kx), J = (int)(cj / d.Ky);
    // near: |I_k - I| <= H and |J_k - J| <= H, as one unsigned range test per axis
    const int Ilo = I - d.H, Jlo = J - d.H;
    const unsigned span = 2u * (unsigned)d.H;
    // keeps r^2 of a lens at the cell centre (always near) away from zero; no
    // effect on any far lens
    const T tiny = PREC != 1 ? (T)1e-300 : (T)1e-30f;
    T zx, zy;
    if (PREC != 1) {
        zx = (T)cell_cx(d, ci);
        zy = (T)cell_cy(d, cj);
    } else {
        zx = (T)cell_cxf(d, ci);
        zy = (T)cell_cyf(d, cj);
    }
    T ar[P], ai[P];
#pragma unroll
    for (int n = 0; n < P; ++n) {
        ar[n] = 0;
        ai[n] = 0;
    }
    for (int64_t base = 0; base < d.nlens; base += kWG) {
        __syncthreads();
        const int64_t k = base + tid;
        if (k < d.nlens) {
            CoefLens<T> L;
            if (PREC != 1) {
                L.x = (T)d.lx[k];
                L.y = (T)d.ly[k];
                L.m = (T)d.lmd[k];
            } else {
                L.x = (T)d.lxf[k];
                L.y = (T)d.lyf[k];
                L.m = (T)d.lmf[k];
            }
            L.I = d.lI[k];
            L.J = d.lJ[k];
            sl[tid] = L;
        }
        __syncthreads();
        const int nb = (int)min((int64_t)kWG, d.nlens - base);
        for (int k2 = 0; k2 < nb; ++k2) {
            const CoefLens<T> L = sl[k2];
            const bool near = ((unsigned)(L.I - Ilo) <= span) & ((unsigned)(L.J - Jlo) <= span);
            T wx = L.x - zx, wy = L.y - zy;
            const T r2 = fma(wx, wx, fma(wy, wy, tiny));
            const T m = near ? (T)0 : L.m;
            // u = 1 / (z_k - z_c) = conj(w) / |w|^2; t = m u^(n+1)
            const T inv = recip_nr2(r2);
            const T ux = wx * inv, uy = -wy * inv;
            T tx = m * ux, ty = m * uy;
#pragma unroll
            for (int n = 0; n < P; ++n) {
                ar[n] -= tx;
                ai[n] -= ty;
                if (n + 1 < P) {
                    const T nx = fma(tx, ux, -(ty * uy));
                    const T ny = fma(tx, uy, ty * ux);
                    tx = nx;
                    ty = ny;
                }
            }
        }
    }
    if (valid) {
        LmCoef& o = out[cj * d.ncx + ci];
        o.a0r = (double)ar[0];
        o.a0i = (double)ai[0];
#pragma unroll
        for (int n = 1; n < 7; ++n) {
            o.a[2 * (n - 1)] = n < P ? (float)ar[n < P ? n : 0] : 0.f;
            o.a[2 * (n - 1) + 1] = n < P ? (float)ai[n < P ? n : 0] : 0.f;
        }
    }
}

// Column offsets dx = local_offset(l) of a level-2 cell and their powers:
// out[k n + l] = dx^(k+1), k < LM_PTAB_POW, and out[LM_PTAB_POW n + l] =
// dx sdx / sdy, l = 0 .. n-1 (entries past R belong
// to masked columns of the last group).
__global__ void k_ptab(LmDesc d, float* __restrict__ out, int n)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < n) {
        float pw[LM_PTAB_POW];
        col_powers<LM_PTAB_POW>(local_offset(l, 0, d.R, d.hxh, d.hxl), pw);
#pragma unroll
        for (int k = 0; k < LM_PTAB_POW; ++k) out[(int64_t)k * n + l] = pw[k];
        out[(int64_t)LM_PTAB_POW * n + l] = pix_ratio(d) * pw[0];
    }
}

// Centre of box (sx, sy) of level-1 cell (I, J) of the hierarchical far
// field: the level-1 cell's centre when it is one box along that axis, else
// the centre of the box's level-2 cells (boxes of d.bx x d.by cells, the last
// one narrower).
__device__ __forceinline__ void box_centre(const LmDesc& d, int64_t I, int64_t J, int sx, int sy,
                                           double& Zx, double& Zy)
{
    if (d.nbx == 1) {
        Zx = d.x0 + ((double)I + 0.5) * (double)((int64_t)d.Kx * d.R) * d.dx;
    } else {
        const int64_t c0 = I * d.Kx + (int64_t)sx * d.bx;
        const int64_t c1 = min(c0 + d.bx, (I + 1) * d.Kx);
        Zx = d.x0 + 0.5 * (double)(c0 + c1) * (double)d.R * d.dx;
    }
    if (d.nby == 1) {
        Zy = d.y0 + ((double)J + 0.5) * (double)((int64_t)d.Ky * d.R) * d.dy;
    } else {
        const int64_t r0 = J * d.Ky + (int64_t)sy * d.by;
        const int64_t r1 = min(r0 + d.by, (J + 1) * d.Ky);
        Zy = d.y0 + 0.5 * (double)(r0 + r1) * (double)d.R * d.dy;
    }
}

// Hierarchical far field, step 1: the series of the far lenses of level-1 cell
// (I, J) about the centre Z of one of its boxes, A_n = -sum_far m_k / (z_k -
// Z)^(n+1), n < Q <= 64 (the level-2 series of Sec. 3.2.2 taken one level up).
// One workgroup per box; the Q terms are cut into ns = ceil(Q / 8) slices of
// eight, and the workgroup's threads into 256 / ns lens groups of ns threads
// (thread s of a group sums terms 8 s .. 8 s + 7 over every (256 / ns)-th far
// lens, so no thread idles on terms past Q); then threads n < Q add the
// groups' partial sums in a fixed order.
__global__ __launch_bounds__(kWG) void k_l1_expand(LmDesc d)
{
    __shared__ double2 part[8 * kWG];  // [groups][8 ns]
    const int ns = (d.Q + 7) >> 3, ng = kWG / ns;
    const int tid = threadIdx.x, grp = tid / ns, s = tid - grp * ns;
    const int64_t cell = blockIdx.x;  // the box: row-major over [n1y nby][n1x nbx]
    const int64_t bi = cell % (d.n1x * d.nbx), bj = cell / (d.n1x * d.nbx);
    const int64_t I = bi / d.nbx, J = bj / d.nby;
    double Zx, Zy;
    box_centre(d, I, J, (int)(bi % d.nbx), (int)(bj % d.nby), Zx, Zy);
    double ar[8], ai[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        ar[j] = 0.0;
        ai[j] = 0.0;
    }
    if (grp < ng) {
        for (int64_t k = grp; k < d.nlens; k += ng) {
            if (abs(d.lI[k] - (int)I) <= d.H && abs(d.lJ[k] - (int)J) <= d.H) continue;
            const double wx = d.lx[k] - Zx, wy = d.ly[k] - Zy;
            const double iw2 = 1.0 / (wx * wx + wy * wy);
            const double ux = wx * iw2, uy = -wy * iw2;  // 1 / (z_k - Z)
            // t = m u^(8 s + 1)
            double px = ux, py = uy;  // u^8 by three squarings
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const double nx = px * px - py * py, ny = 2.0 * px * py;
                px = nx;
                py = ny;
            }
            double tx = d.lmd[k] * ux, ty = d.lmd[k] * uy;
            for (int q = 0; q < s; ++q) {
                const double nx = tx * px - ty * py, ny = tx * py + ty * px;
                tx = nx;
                ty = ny;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                ar[j] -= tx;
                ai[j] -= ty;
                const double nx = tx * ux - ty * uy, ny = tx * uy + ty * ux;
                tx = nx;
                ty = ny;
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) part[8 * tid + j] = make_double2(ar[j], ai[j]);
    }
    __syncthreads();
    if (tid < d.Q) {
        // term n of group g sits at 8 (g ns + n / 8) + n % 8 = 8 g ns + n
        double sr = 0.0, si = 0.0;
        for (int g = 0; g < ng; ++g) {
            sr += part[8 * ns * g + tid].x;
            si += part[8 * ns * g + tid].y;
        }
        d.l1exp[2 * (cell * d.Q + tid)] = sr;
        d.l1exp[2 * (cell * d.Q + tid) + 1] = si;
    }
}

// Hierarchical far field, step 2: the series of step 1 of the box holding each
// level-2 cell re-expanded about the cell's centre z_c, a_p = sum_{n>=p}
// C(n,p) A_n (z_c - Z)^(n-p), with T_n[p] = C(n,p) w^(n-p) advanced by
// T_{n+1}[p] = w T_n[p] + T_n[p-1].
template <int P>
__global__ __launch_bounds__(kWG) void k_l1_shift(LmDesc d, LmCoef* __restrict__ out)
{
    const int64_t c = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (c >= d.ncx * d.ncy) return;
    const int64_t ci = c % d.ncx, cj = c / d.ncx;
    const int64_t I = ci / d.Kx, J = cj / d.Ky;
    const int sx = (int)((ci - I * d.Kx) / d.bx), sy = (int)((cj - J * d.Ky) / d.by);
    double Zx, Zy;
    box_centre(d, I, J, sx, sy, Zx, Zy);
    const int64_t box = (J * d.nby + sy) * (d.n1x * d.nbx) + (I * d.nbx + sx);
    const double wx = cell_cx(d, ci) - Zx, wy = cell_cy(d, cj) - Zy;
    double tr[P], ti[P], ar[P], ai[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        tr[p] = p == 0 ? 1.0 : 0.0;
        ti[p] = 0.0;
        ar[p] = 0.0;
        ai[p] = 0.0;
    }
    const double* A = d.l1exp + 2 * (box * d.Q);
    for (int n = 0; n < d.Q; ++n) {
        const double Ar = A[2 * n], Ai = A[2 * n + 1];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            ar[p] += Ar * tr[p] - Ai * ti[p];
            ai[p] += Ar * ti[p] + Ai * tr[p];
        }
#pragma unroll
        for (int p = P - 1; p >= 0; --p) {
            const double nr = tr[p] * wx - ti[p] * wy + (p > 0 ? tr[p > 0 ? p - 1 : 0] : 0.0);
            const double ni = tr[p] * wy + ti[p] * wx + (p > 0 ? ti[p > 0 ? p - 1 : 0] : 0.0);
            tr[p] = nr;
            ti[p] = ni;
        }
    }
    LmCoef& o = out[cj * d.ncx + ci];
    o.a0r = ar[0];
    o.a0i = ai[0];
#pragma unroll
    for (int n = 1; n < 7; ++n) {
        o.a[2 * (n - 1)] = n < P ? (float)ar[n < P ? n : 0] : 0.f;
        o.a[2 * (n - 1) + 1] = n < P ? (float)ai[n < P ? n : 0] : 0.f;
    }
}

__global__ __launch_bounds__(kWG) void k_sum_u64(const unsigned long long* __restrict__ p,
                                                 int64_t n, unsigned long long* total)
{
    unsigned long long s = 0;
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWG)
        s += p[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(total, s);
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Rows [q0, q0 + nq) x columns [p0, p0 + np) of a row-major map of width snx,
// packed row after row into out (np * nq values).
__global__ void k_copy_region_u64(const unsigned long long* __restrict__ map, int64_t snx,
                                  int64_t p0, int64_t q0, int64_t np, int64_t n,
                                  unsigned long long* __restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / np, c = i - r * np;
        out[i] = map[(q0 + r) * snx + p0 + c];
    }
}

// ------------------------------------------------ the rectangle sheet

struct Cd {
    double r, i;
};
__device__ __forceinline__ Cd cd(double r, double i) { return Cd{r, i}; }
__device__ __forceinline__ Cd operator+(Cd a, Cd b) { return cd(a.r + b.r, a.i + b.i); }
__device__ __forceinline__ Cd operator-(Cd a, Cd b) { return cd(a.r - b.r, a.i - b.i); }
__device__ __forceinline__ Cd operator*(Cd a, Cd b)
{
    return cd(a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r);
}
__device__ __forceinline__ Cd operator*(double s, Cd a) { return cd(s * a.r, s * a.i); }
__device__ __forceinline__ Cd cinv(Cd a)
{
    const double n = a.r * a.r + a.i * a.i;
    return cd(a.r / n, -a.i / n);
}
// principal logarithm of wq / wp
__device__ __forceinline__ Cd clog_ratio(Cd wq, Cd wp)
{
    const double qr = wq.r * wp.r + wq.i * wp.i, qi = wq.i * wp.r - wq.r * wp.i;
    const double nq = wq.r * wq.r + wq.i * wq.i, np = wp.r * wp.r + wp.i * wp.i;
    return cd(0.5 * log(nq / np), atan2(qi, qr));
}

// The sheet of density -kappa_star on the lenses' rectangle (Sec. 2, Eq. 6):
// inside the rectangle its term in the lens equation is kappa_star theta +
// h(theta), and by Green's theorem on the rectangle
//   conj(h)(z) = (kappa_star / 2 pi i) oint z'* / (z - z') dz'
// over its edges, counter-clockwise.  About an expansion point z_e inside,
// conj(h) = sum_n H_n (z - z_e)^n with H_n = -(kappa_star / 2 pi i) J_n,
//   J_n = oint z'* w^-(n+1) dz',  w = z' - z_e.
// On an edge z'* is linear in z' (y = y_e: z'* = z' - 2 i y_e; x = x_e:
// z'* = 2 x_e - z'), so z'* = s w + c there and each edge from wP to wQ gives
//   n = 0:  s (wQ - wP) + c Log(wQ / wP)
//   n = 1:  s Log(wQ / wP) + c (1/wP - 1/wQ)
//   n >= 2: s (wQ^(1-n) - wP^(1-n)) / (1 - n) + c (wP^-n - wQ^-n) / n
// (a straight edge that misses z_e turns by less than pi about it, so the
// principal logarithm of the ratio is the integral).  The far field enters the
// lens equation as -alpha_far with conj(alpha_far) = sum a_n delta^n and the
// sheet as +h, so a_n gains -H_n = (kappa_star / 2 pi i) J_n.  z_e is the
// centre of the part of the cell inside the lattice (the cell centre except
// in a partial last column or row), and the polynomial is re-expanded about
// the cell centre: b'_k = sum_{n>=k} C(n,k) b_n t^(n-k), t = z_c - z_e.
template <int P>
__global__ __launch_bounds__(kWG) void k_sheet(LmDesc d, LmCoef* __restrict__ out)
{
    const int64_t c = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (c >= d.ncx * d.ncy) return;
    const int64_t ci = c % d.ncx, cj = c / d.ncx;
    const int64_t i1 = min((ci + 1) * (int64_t)d.R, d.nx), j1 = min((cj + 1) * (int64_t)d.R, d.ny);
    const Cd ze = cd(d.x0 + 0.5 * ((double)(ci * d.R) + (double)i1) * d.dx,
                     d.y0 + 0.5 * ((double)(cj * d.R) + (double)j1) * d.dy);
    const Cd corner[4] = {cd(d.sx0, d.sy0), cd(d.sx1, d.sy0), cd(d.sx1, d.sy1),
                          cd(d.sx0, d.sy1)};
    // z'* = s w + c on the four edges, counter-clockwise from (sx0, sy0)
    const double es[4] = {1.0, -1.0, 1.0, -1.0};
    const Cd ec[4] = {ze - cd(0.0, 2.0 * d.sy0), cd(2.0 * d.sx1, 0.0) - ze,
                      ze - cd(0.0, 2.0 * d.sy1), cd(2.0 * d.sx0, 0.0) - ze};
    Cd J[P];
#pragma unroll
    for (int n = 0; n < P; ++n) J[n] = cd(0.0, 0.0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const Cd wp = corner[e] - ze, wq = corner[(e + 1) & 3] - ze;
        const double s = es[e];
        const Cd cc = ec[e];
        const Cd L = clog_ratio(wq, wp);
        const Cd ip = cinv(wp), iq = cinv(wq);
        J[0] = J[0] + s * (wq - wp) + cc * L;
        if constexpr (P > 1) J[1] = J[1] + s * L + cc * (ip - iq);
        // wP^-(n-1), wQ^-(n-1) and wP^-n, wQ^-n, advanced by one power per n
        Cd pp = ip, pq = iq, p2 = ip * ip, q2 = iq * iq;
#pragma unroll
        for (int n = 2; n < P; ++n) {
            J[n] = J[n] + (s / (1.0 - n)) * (pq - pp) + (1.0 / n) * (cc * (p2 - q2));
            pp = p2;
            pq = q2;
            p2 = p2 * ip;
            q2 = q2 * iq;
        }
    }
    // b_n = (kappa_star / 2 pi i) J_n = (kappa_star / 2 pi) (Im J_n, -Re J_n)
    const double f = d.kappa_star / (2.0 * 3.14159265358979323846);
    Cd b[P];
#pragma unroll
    for (int n = 0; n < P; ++n) b[n] = cd(f * J[n].i, -f * J[n].r);
    const Cd t = cd(cell_cx(d, ci), cell_cy(d, cj)) - ze;
    LmCoef& o = out[cj * d.ncx + ci];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        Cd acc = cd(0.0, 0.0), tp = cd(1.0, 0.0);
        double binom = 1.0;
#pragma unroll
        for (int n = k; n < P; ++n) {
            acc = acc + binom * (b[n] * tp);
            tp = tp * t;
            binom = binom * (double)(n + 1) / (double)(n + 1 - k);
        }
        if (k == 0) {
            o.a0r += acc.r;
            o.a0i += acc.i;
        } else {
            o.a[2 * k - 2] = (float)((double)o.a[2 * k - 2] + acc.r);
            o.a[2 * k - 1] = (float)((double)o.a[2 * k - 1] + acc.i);
        }
    }
}

// Near-lens deflection of each level-2 cell centre, one cell per thread: the
// sum over the cell's near list, in list order, of m (z_c - z_k) / |z_c - z_k|^2
// in FP64 (the centred near sums add each ray's FP32 change from it).  NaN when
// a near lens lies within twice the cell's half-diagonal of the centre: there
// the change is not small, and the shooting kernel sums that cell's near
// lenses plainly.
__global__ __launch_bounds__(kWG) void k_near_centre(LmDesc d, LmCoef* __restrict__ out)
{
    const int64_t c = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (c >= d.ncx * d.ncy) return;
    const int64_t ci = c % d.ncx, cj = c / d.ncx;
    const double zcx = cell_cx(d, ci), zcy = cell_cy(d, cj);
    const double rc2 = (double)d.R * d.R * (d.dx * d.dx + d.dy * d.dy);
    const L1Cell l1 = l1_of(d, ci, cj);
    double sx = 0.0, sy = 0.0;
    bool close = false;
    for (int r = 0; r <= 2 * d.H; ++r) {
        int s, e;
        near_row(d, l1, r, s, e);
        for (int k = s; k < e; ++k) {
            const double ox = d.lx[k] - zcx, oy = d.ly[k] - zcy;
            const double r2 = ox * ox + oy * oy;
            close |= r2 < rc2;
            const double q = d.lmd[k] / r2;
            sx -= q * ox;
            sy -= q * oy;
        }
    }
    LmCoef& o = out[cj * d.ncx + ci];
    o.n0x = close ? __builtin_nan("") : sx;
    o.n0y = close ? __builtin_nan("") : sy;
}

}  // namespace

// Every (scheme, precision) pair lm_shoot_inst.hip is built for.
#define LM_PAIRS(X) X(0, 0) X(0, 1) X(1, 0) X(1, 1) X(1, 2) X(1, 4)

bool lm_supported_rays_per_lane(int r) { return r == 4 || r == 8 || r == 16; }

int lm_launch_shoot_map(const LmDesc& d, int scheme, int precision, int terms, int rays_per_lane,
                        void* stream)
{
    if (d.ntiles <= 0) return 0;
#define X(S, PR)                                                                            \
    if (scheme == S && precision == PR)                                                     \
        return LM_INST_CAT(lm_inst_shoot_map, S, PR)(d, rays_per_lane, terms, stream);
    LM_PAIRS(X)
#undef X
    return (int)hipErrorInvalidValue;
}

int lm_launch_shoot_batch(const LmDesc* descs, const int64_t* offsets, const int32_t* order,
                          int nmaps, unsigned long long* queue, int scheme, int precision,
                          int terms, int rays_per_lane, int layout, int grid, void* stream)
{
#define X(S, PR)                                                                            \
    if (scheme == S && precision == PR)                                                     \
        return LM_INST_CAT(lm_inst_shoot_batch, S, PR)(descs, offsets, order, nmaps, queue, \
                                                       rays_per_lane, terms, layout, grid,  \
                                                       stream);
    LM_PAIRS(X)
#undef X
    return (int)hipErrorInvalidValue;
}

int lm_shoot_occupancy(int scheme, int precision, int terms, int rays_per_lane, int layout,
                       int* wg_per_cu)
{
#define X(S, PR)                                                                            \
    if (scheme == S && precision == PR)                                                     \
        return LM_INST_CAT(lm_inst_occupancy, S, PR)(rays_per_lane, terms, layout, wg_per_cu);
    LM_PAIRS(X)
#undef X
    return (int)hipErrorInvalidValue;
}

int lm_launch_trace(const LmDesc& d, int scheme, int precision, int terms, const int64_t* ii,
                    const int64_t* jj, int64_t n, int32_t* p, int32_t* q, double* uv,
                    void* stream)
{
    if (n <= 0) return 0;
#define X(S, PR)                                                                            \
    if (scheme == S && precision == PR)                                                     \
        return LM_INST_CAT(lm_inst_trace, S, PR)(d, terms, ii, jj, n, p, q, uv, stream);
    LM_PAIRS(X)
#undef X
    return (int)hipErrorInvalidValue;
}

int lm_launch_deflect(const LmDesc& d, int scheme, int precision, int terms, const double* th,
                      int64_t n, double* alpha, void* stream)
{
    if (n <= 0) return 0;
#define X(S, PR)                                                                            \
    if (scheme == S && precision == PR)                                                     \
        return LM_INST_CAT(lm_inst_deflect, S, PR)(d, terms, th, n, alpha, stream);
    LM_PAIRS(X)
#undef X
    return (int)hipErrorInvalidValue;
}

int lm_launch_coeffs_hier(const LmDesc& d, int terms, LmCoef* out, void* stream)
{
    const int64_t n1 = d.n1x * d.nbx * d.n1y * d.nby, n2 = d.ncx * d.ncy;
    if (n1 <= 0 || n2 <= 0) return 0;
    if (d.Q < terms || d.Q > 64) return (int)hipErrorInvalidValue;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_l1_expand, dim3((unsigned)n1), dim3(kWG), 0, s, d);
    const int e = (int)hipGetLastError();
    if (e) return e;
    const dim3 grid((unsigned)((n2 + kWG - 1) / kWG));
    switch (terms) {
    case 1: hipLaunchKernelGGL(k_l1_shift<1>, grid, dim3(kWG), 0, s, d, out); break;
    case 2: hipLaunchKernelGGL(k_l1_shift<2>, grid, dim3(kWG), 0, s, d, out); break;
    case 3: hipLaunchKernelGGL(k_l1_shift<3>, grid, dim3(kWG), 0, s, d, out); break;
    case 4: hipLaunchKernelGGL(k_l1_shift<4>, grid, dim3(kWG), 0, s, d, out); break;
    case 5: hipLaunchKernelGGL(k_l1_shift<5>, grid, dim3(kWG), 0, s, d, out); break;
    case 6: hipLaunchKernelGGL(k_l1_shift<6>, grid, dim3(kWG), 0, s, d, out); break;
    case 7: hipLaunchKernelGGL(k_l1_shift<7>, grid, dim3(kWG), 0, s, d, out); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int lm_launch_sheet(const LmDesc& d, int terms, LmCoef* coef, void* stream)
{
    const int64_t n = d.ncx * d.ncy;
    if (n <= 0 || !d.sheet) return 0;
    const dim3 grid((unsigned)((n + kWG - 1) / kWG));
    hipStream_t s = (hipStream_t)stream;
    switch (terms) {
    case 1: hipLaunchKernelGGL(k_sheet<1>, grid, dim3(kWG), 0, s, d, coef); break;
    case 2: hipLaunchKernelGGL(k_sheet<2>, grid, dim3(kWG), 0, s, d, coef); break;
    case 3: hipLaunchKernelGGL(k_sheet<3>, grid, dim3(kWG), 0, s, d, coef); break;
    case 4: hipLaunchKernelGGL(k_sheet<4>, grid, dim3(kWG), 0, s, d, coef); break;
    case 5: hipLaunchKernelGGL(k_sheet<5>, grid, dim3(kWG), 0, s, d, coef); break;
    case 6: hipLaunchKernelGGL(k_sheet<6>, grid, dim3(kWG), 0, s, d, coef); break;
    case 7: hipLaunchKernelGGL(k_sheet<7>, grid, dim3(kWG), 0, s, d, coef); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int lm_launch_near_centre(const LmDesc& d, LmCoef* out, void* stream)
{
    const int64_t n = d.ncx * d.ncy;
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_near_centre, dim3((unsigned)((n + kWG - 1) / kWG)), dim3(kWG), 0,
                       (hipStream_t)stream, d, out);
    return (int)hipGetLastError();
}

int lm_launch_ptab(const LmDesc& d, float* out, int n, void* stream)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_ptab, dim3((unsigned)((n + kWG - 1) / kWG)), dim3(kWG), 0,
                       (hipStream_t)stream, d, out, n);
    return (int)hipGetLastError();
}

int lm_launch_sum_u64(const unsigned long long* p, int64_t n, unsigned long long* total,
                      void* stream)
{
    if (n <= 0) return 0;
    int64_t blocks = (n + kWG - 1) / kWG;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_sum_u64, dim3((unsigned)blocks), dim3(kWG), 0, (hipStream_t)stream, p, n,
                       total);
    return (int)hipGetLastError();
}

int lm_launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, void* stream)
{
    if (n <= 0) return 0;
    int64_t blocks = (n + kWG - 1) / kWG;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(kWG), 0, (hipStream_t)stream, p, n,
                       v);
    return (int)hipGetLastError();
}

int lm_launch_copy_region_u64(const unsigned long long* map, int64_t snx, int64_t p0, int64_t q0,
                              int64_t np, int64_t nq, unsigned long long* out, void* stream)
{
    const int64_t n = np * nq;
    if (n <= 0) return 0;
    int64_t blocks = (n + kWG - 1) / kWG;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_copy_region_u64, dim3((unsigned)blocks), dim3(kWG), 0,
                       (hipStream_t)stream, map, snx, p0, q0, np, n, out);
    return (int)hipGetLastError();
}

int lm_launch_coeffs(const LmDesc& d, int precision, int terms, int64_t ci0, int64_t cj0,
                     int64_t nci, int64_t ncj, LmCoef* out, void* stream)
{
    const int64_t n = nci * ncj;
    if (n <= 0) return 0;
    const dim3 grid((unsigned)((n + kWG - 1) / kWG));
    hipStream_t s = (hipStream_t)stream;
#define LM_COEF(PR, P) \
    hipLaunchKernelGGL((k_coeffs<PR, P>), grid, dim3(kWG), 0, s, d, ci0, cj0, nci, ncj, out)
#define LM_COEF_P(PR)                         \
    switch (terms) {                          \
    case 1: LM_COEF(PR, 1); break;            \
    case 2: LM_COEF(PR, 2); break;            \
    case 3: LM_COEF(PR, 3); break;            \
    case 4: LM_COEF(PR, 4); break;            \
    case 5: LM_COEF(PR, 5); break;            \
    case 6: LM_COEF(PR, 6); break;            \
    case 7: LM_COEF(PR, 7); break;            \
    default: return (int)hipErrorInvalidValue; \
    }
    if (precision != 1) {
        LM_COEF_P(0)
    } else {
        LM_COEF_P(1)
    }
#undef LM_COEF_P
#undef LM_COEF
    return (int)hipGetLastError();
}
