// Spreading onto and gathering from the oversampled grid (the paper's
// "diffusion" of the point data to the regular grid X through a smooth,
// localized window), with a Kaiser-Bessel window.
//
// Window (grid-cell units, normalized by I0(m b)); the FP32 path evaluates the
// taps as degree-7 polynomials of the in-cell fraction fitted at plan time (max
// error 8e-8 of the peak, below the closed form's FP32 rounding):
//   psi(t) = (e^{-b t^2/(z + m)} - e^{-b (z + m)}) / (2 pi z I0e(m b)),  z = sqrt(m^2 - t^2), |t| < m
// which equals sinh(b z) / (pi z I0(m b)); zero for |t| >= m.  A point with grid
// coordinate u has taps k = floor(u) - m + 1 + a, a = 0..2m-1, at t = u - k.
//
// Spread: one workgroup per T x T tile of base cells (T = 16 or 32, a run-time shape:
// smaller tiles make more workgroups for small grids).  Every wave owns a
// private FP64 accumulator for the padded tile (T + 2m - 1 cells a side) in
// LDS; the window products (FP32 or FP64) are added with LDS atomics that only
// that wave touches, so the summation order is fixed and no global atomics are
// used.  The wave copies are summed in a fixed order into a per-tile buffer, and
// fold() adds the (at most four) padded tiles covering each cell.
//
// Gather: one workgroup per tile; the padded grid tile of every field is staged
// in LDS; each thread takes one target: rows of 2m taps are summed in the grid
// precision, the 2m row sums are accumulated in FP64.
#include "fn_internal.h"

#include <type_traits>

namespace fn {

namespace {

#ifndef FN_SPREAD_CELLS
#define FN_SPREAD_CELLS 1  // mixed path: one thread per grid cell (k_spread_cells)
#endif
constexpr int SPREAD_WAVES = 2;
constexpr uint32_t SPREAD_FLUSH = 8;  // points per FP32 register sum in k_spread_cells
constexpr int SPREAD_NT = 64 * SPREAD_WAVES;

// z - m is formed as -t^2/(z + m): for the central taps z is close to m and the
// direct difference would lose most of the FP32 mantissa.
template <typename R>
__device__ __forceinline__ R kb_psi(R t, R m, R b, R wnorm)
{
    const R t2 = t * t;
    const R z2 = m * m - t2;
    if (!(z2 > (R)0)) return (R)0;
    const R z = sqrt(z2);
    const R zm = z + m;
    return (exp(-b * t2 / zm) - exp(-b * zm)) * wnorm / z;
}

// The 2m taps of the window at fraction f into w[]: the FP32 path evaluates the
// tap polynomials (taps a and 2m-1-a from one even/odd pair in u = 2f - 1, the
// coefficients uniform across the wave), the FP64 path the closed form.
template <typename R, int M2>
__device__ __forceinline__ void taps(const WinPoly &wp, R f, R rm, R rb, R rw, R (&w)[M2])
{
    constexpr int m = M2 / 2;
    if (sizeof(R) == 4) {
        const float u = fmaf(2.0f, (float)f, -1.0f);
        const float v = u * u;
#pragma unroll
        for (int a = 0; a < m; ++a) {
            const float e = fmaf(fmaf(fmaf(wp.c[a][3], v, wp.c[a][2]), v, wp.c[a][1]), v, wp.c[a][0]);
            const float o = fmaf(fmaf(fmaf(wp.c[a][7], v, wp.c[a][6]), v, wp.c[a][5]), v, wp.c[a][4]);
            w[a] = (R)fmaf(u, o, e);
            w[M2 - 1 - a] = (R)fmaf(-u, o, e);
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < M2; ++a) w[a] = kb_psi<R>(f + (R)(m - 1 - a), rm, rb, rw);
}

template <typename R> __device__ __forceinline__ R frac_of(const float *f32, const double *f64, int64_t i);
template <> __device__ __forceinline__ float frac_of<float>(const float *f32, const double *, int64_t i)
{
    return f32[i];
}
template <> __device__ __forceinline__ double frac_of<double>(const float *, const double *f64, int64_t i)
{
    return f64[i];
}

// rows [y0, y0 + TL) x cells [x0, x1) of a cell-sorted point set: per-row start and prefix
template <int TL>
struct TileRows {
    uint32_t start[TL];
    uint32_t pre[TL + 1];
};

template <int TL>
__device__ __forceinline__ void tile_rows(TileRows<TL> &tr, const uint32_t *__restrict__ cstart, int Ex, int Ey,
                                          int x0, int y0)
{
    const int x1 = min(x0 + TL, Ex);
    if (threadIdx.x < TL) {
        const int y = y0 + threadIdx.x;
        uint32_t s = 0, e = 0;
        if (y < Ey) {
            s = cstart[(int64_t)y * Ex + x0];
            e = cstart[(int64_t)y * Ex + x1];
        }
        tr.start[threadIdx.x] = s;
        tr.pre[threadIdx.x + 1] = e - s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        tr.pre[0] = 0;
        for (int r = 1; r <= TL; ++r) tr.pre[r] += tr.pre[r - 1];
    }
    __syncthreads();
}

template <int TL>
__device__ __forceinline__ int64_t tile_point(const TileRows<TL> &tr, uint32_t k)
{
    int lo = 0, hi = TL - 1;  // largest r with pre[r] <= k
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (tr.pre[mid] <= k) lo = mid; else hi = mid - 1;
    }
    return (int64_t)tr.start[lo] + (k - tr.pre[lo]);
}

template <typename R, int M2, int TL>
__global__ void __launch_bounds__(SPREAD_NT) k_spread(const uint32_t *__restrict__ key, const float *__restrict__ fr32,
                                                      const double *__restrict__ fr64, const R *__restrict__ val,
                                                      int64_t N, const uint32_t *__restrict__ cstart, int Ex, int Ey,
                                                      int ntx, int nty, double b, double wnorm, int nfield,
                                                      double *__restrict__ ptile, const WinPoly wp)
{
    constexpr int m = M2 / 2;
    constexpr int PT = TL + M2 - 1;
    constexpr int PT2 = PT * PT;
    extern __shared__ double acc[];  // [SPREAD_WAVES][nfield][PT2]
    __shared__ TileRows<TL> tr;
    const int tile = blockIdx.x;
    const int tx = tile % ntx, ty = tile / ntx;
    const int x0 = tx * TL, y0 = ty * TL;
    const int wv = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < SPREAD_WAVES * nfield * PT2; i += SPREAD_NT) acc[i] = 0.0;
    tile_rows(tr, cstart, Ex, Ey, x0, y0);
    const uint32_t P = tr.pre[TL];
    double *myacc = acc + (int64_t)wv * nfield * PT2;
    const R rm = (R)m, rb = (R)b, rw = (R)wnorm;
    for (uint32_t k = threadIdx.x; k < P; k += SPREAD_NT) {
        const int64_t i = tile_point(tr, k);
        const uint32_t kk = key[i];
        const int lx = (int)(kk % (uint32_t)Ex) - x0, ly = (int)(kk / (uint32_t)Ex) - y0;
        const R fx = frac_of<R>(fr32, fr64, i), fy = frac_of<R>(fr32, fr64, N + i);
        R wx[M2], wy[M2];
        taps<R, M2>(wp, fx, rm, rb, rw, wx);
        taps<R, M2>(wp, fy, rm, rb, rw, wy);
        for (int f = 0; f < nfield; ++f) {
            const R v = val[(int64_t)f * N + i];
            double *af = myacc + f * PT2 + ly * PT + lx;
#pragma unroll
            for (int bb = 0; bb < M2; ++bb) {
                const R vy = v * wy[bb];
#pragma unroll
                for (int a = 0; a < M2; ++a) atomicAdd(af + bb * PT + a, (double)(vy * wx[a]));
            }
        }
    }
    __syncthreads();
    const int ntiles = ntx * nty;
    for (int f = 0; f < nfield; ++f)
        for (int c = threadIdx.x; c < PT2; c += SPREAD_NT) {
            double v = acc[f * PT2 + c];
            for (int w = 1; w < SPREAD_WAVES; ++w) v += acc[((int64_t)w * nfield + f) * PT2 + c];
            ptile[((int64_t)f * ntiles + tile) * PT2 + c] = v;
        }
}

// Taps a and 2m-1-a (a < m) of the FP32 tap polynomials at u = 2f - 1, v = u^2.
__device__ __forceinline__ void tap_pair(const WinPoly &wp, int a, float u, float v, float &lo, float &hi)
{
    const float e = fmaf(fmaf(fmaf(wp.c[a][3], v, wp.c[a][2]), v, wp.c[a][1]), v, wp.c[a][0]);
    const float o = fmaf(fmaf(fmaf(wp.c[a][7], v, wp.c[a][6]), v, wp.c[a][5]), v, wp.c[a][4]);
    lo = fmaf(u, o, e);
    hi = fmaf(-u, o, e);
}

// Mixed-precision spread, one thread per grid cell: the points of a cell share one
// 2m x 2m footprint, so their window products are summed in FP32 registers (a
// handful of terms) and added to the wave's FP64 accumulator once per cell.  The
// footprint's rows are taken in NG groups, each holding whole row pairs (a, 2m-1-a):
// a pair of y taps comes from one even/odd polynomial pair, so every y tap is evaluated
// once per point whatever NG is; the x taps are evaluated once per group.  NG = 1 keeps
// all 4m^2 sums in registers.  The lanes of a wave hold consecutive cells of a tile row,
// so every LDS atomic instruction touches consecutive addresses.  Same accumulator layout
// and fixed per-wave summation order as k_spread.
template <int M2, int NG, int TL>
__global__ void __launch_bounds__(SPREAD_NT) k_spread_cells(const float *__restrict__ fr32,
                                                            const float *__restrict__ val, int64_t N,
                                                            const uint32_t *__restrict__ cstart, int Ex, int Ey,
                                                            int ntx, int nty, double *__restrict__ ptile,
                                                            const WinPoly wp)
{
    constexpr int m = M2 / 2;
    constexpr int PT = TL + M2 - 1;
    constexpr int PT2 = PT * PT;
    constexpr int PPG = (m + NG - 1) / NG;  // row pairs per group
    extern __shared__ double acc[];  // [SPREAD_WAVES][PT2]
    // one block per (field, tile): a block's LDS holds one field, so a two-field
    // spread keeps the occupancy of a one-field one
    const int ntiles = ntx * nty;
    const int f = blockIdx.x / ntiles;
    const int tile = blockIdx.x - f * ntiles;
    const int tx = tile % ntx, ty = tile / ntx;
    const int x0 = tx * TL, y0 = ty * TL;
    const int wv = threadIdx.x >> 6;
    // an empty tile (a sparse point set) only writes its zero partial sums
    __shared__ int tile_pts;
    if (threadIdx.x == 0) tile_pts = 0;
    __syncthreads();
    if (threadIdx.x < TL && y0 + (int)threadIdx.x < Ey && x0 < Ex) {
        const int64_t rb = (int64_t)(y0 + threadIdx.x) * Ex;
        if (cstart[rb + min(x0 + TL, Ex)] != cstart[rb + x0]) atomicOr(&tile_pts, 1);
    }
    __syncthreads();
    if (tile_pts == 0) {  // uniform
        for (int c = threadIdx.x; c < PT2; c += SPREAD_NT) ptile[((int64_t)f * ntiles + tile) * PT2 + c] = 0.0;
        return;
    }
    for (int i = threadIdx.x; i < SPREAD_WAVES * PT2; i += SPREAD_NT) acc[i] = 0.0;
    __syncthreads();
    double *myacc = acc + (int64_t)wv * PT2;
    const float *fval = val + (int64_t)f * N;
    // point range of cell c of the tile (empty outside the grid)
    auto cell_range = [&](int c, uint32_t &a, uint32_t &b) {
        const int gx = x0 + c % TL, gy = y0 + c / TL;
        a = b = 0;
        if (c < TL * TL && gx < Ex && gy < Ey) {
            const int64_t cell = (int64_t)gy * Ex + gx;
            a = cstart[cell];
            b = cstart[cell + 1];
        }
    };
    uint32_t n0, n1;
    cell_range(threadIdx.x, n0, n1);
    for (int c = threadIdx.x; c < TL * TL; c += SPREAD_NT) {
        const int lx = c % TL, ly = c / TL;
        const uint32_t s0 = n0, s1 = n1;
        cell_range(c + SPREAD_NT, n0, n1);  // the next cell's range loads while this one runs
        if (s0 == s1) continue;
        // at most SPREAD_FLUSH points per FP32 register sum, then into the FP64 accumulator
        // (a dense cluster can put thousands of points in one cell)
        for (uint32_t i0 = s0; i0 < s1; i0 += SPREAD_FLUSH) {
            const uint32_t i1 = min(s1, i0 + SPREAD_FLUSH);
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int a0 = g * PPG;  // first row pair of the group
                // r[2k] is row a0 + k, r[2k + 1] is row 2m - 1 - (a0 + k)
                float r[2 * PPG][M2];
#pragma unroll
                for (int k = 0; k < 2 * PPG; ++k)
#pragma unroll
                    for (int a = 0; a < M2; ++a) r[k][a] = 0.f;
                for (uint32_t i = i0; i < i1; ++i) {
                    const float v = fval[i];
                    float wx[M2];
                    taps<float, M2>(wp, fr32[i], 0.f, 0.f, 0.f, wx);
                    const float uy = fmaf(2.0f, fr32[N + i], -1.0f), vy2 = uy * uy;
#pragma unroll
                    for (int k = 0; k < PPG; ++k) {
                        if (a0 + k >= m) break;
                        float ylo, yhi;
                        tap_pair(wp, a0 + k, uy, vy2, ylo, yhi);
                        const float vl = v * ylo, vh = v * yhi;
#pragma unroll
                        for (int a = 0; a < M2; ++a) {
                            r[2 * k][a] = fmaf(vl, wx[a], r[2 * k][a]);
                            r[2 * k + 1][a] = fmaf(vh, wx[a], r[2 * k + 1][a]);
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < PPG; ++k) {
                    if (a0 + k >= m) break;
                    double *alo = myacc + (ly + a0 + k) * PT + lx;
                    double *ahi = myacc + (ly + M2 - 1 - (a0 + k)) * PT + lx;
#pragma unroll
                    for (int a = 0; a < M2; ++a) atomicAdd(alo + a, (double)r[2 * k][a]);
#pragma unroll
                    for (int a = 0; a < M2; ++a) atomicAdd(ahi + a, (double)r[2 * k + 1][a]);
                }
            }
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < PT2; c += SPREAD_NT) {
        double v = acc[c];
        for (int w = 1; w < SPREAD_WAVES; ++w) v += acc[(int64_t)w * PT2 + c];
        ptile[((int64_t)f * ntiles + tile) * PT2 + c] = v;
    }
}

template <typename R>
__global__ void k_fold(const double *__restrict__ ptile, int Ex, int Ey, int ntx, int nty, int TILE, int PT, int nfield,
                       R *__restrict__ grid, int64_t fstride)
{
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)Ex * Ey) return;
    const int X = (int)(idx % Ex), Y = (int)(idx / Ex);
    const int tx = X / TILE, ty = Y / TILE, lx = X % TILE, ly = Y % TILE;
    const int64_t ntiles = (int64_t)ntx * nty, PT2 = (int64_t)PT * PT;
    for (int f = 0; f < nfield; ++f) {
        const double *pf = ptile + f * ntiles * PT2;
        double v = pf[((int64_t)ty * ntx + tx) * PT2 + ly * PT + lx];
        const bool left = tx > 0 && lx + TILE < PT, down = ty > 0 && ly + TILE < PT;
        if (left) v += pf[((int64_t)ty * ntx + tx - 1) * PT2 + ly * PT + lx + TILE];
        if (down) v += pf[((int64_t)(ty - 1) * ntx + tx) * PT2 + (ly + TILE) * PT + lx];
        if (left && down) v += pf[((int64_t)(ty - 1) * ntx + tx - 1) * PT2 + (ly + TILE) * PT + lx + TILE];
        grid[f * fstride + idx] = (R)v;
    }
}

template <typename R, int M2, int TL>
__global__ void __launch_bounds__(256) k_gather(const uint32_t *__restrict__ key, const float *__restrict__ fr32,
                                                const double *__restrict__ fr64, int64_t N,
                                                const uint32_t *__restrict__ cstart, int Ex, int Ey, int ntx,
                                                double b, double wnorm, const R *__restrict__ grid,
                                                int64_t fstride, int nfield, double *__restrict__ far,
                                                int64_t farstride, const WinPoly wp)
{
    constexpr int m = M2 / 2;
    constexpr int PT = TL + M2 - 1;
    constexpr int PT2 = PT * PT;
    extern __shared__ char smem_g[];
    R *L = reinterpret_cast<R *>(smem_g);  // [nfield][PT2]
    __shared__ TileRows<TL> tr;
    const int tile = blockIdx.x;
    const int tx = tile % ntx, ty = tile / ntx;
    const int x0 = tx * TL, y0 = ty * TL;
    tile_rows(tr, cstart, Ex, Ey, x0, y0);
    const uint32_t P = tr.pre[TL];
    if (P == 0) return;  // uniform across the block
    for (int f = 0; f < nfield; ++f)
        for (int c = threadIdx.x; c < PT2; c += blockDim.x) {
            const int X = x0 + c % PT, Y = y0 + c / PT;
            L[f * PT2 + c] = (X < Ex && Y < Ey) ? grid[f * fstride + (int64_t)Y * Ex + X] : (R)0;
        }
    __syncthreads();
    const R rm = (R)m, rb = (R)b, rw = (R)wnorm;
    // the next target's cell and fractions load while this one is summed
    int64_t ni = 0;
    uint32_t nk = 0;
    R nfx = (R)0, nfy = (R)0;
    if (threadIdx.x < P) {
        ni = tile_point(tr, threadIdx.x);
        nk = key[ni];
        nfx = frac_of<R>(fr32, fr64, ni);
        nfy = frac_of<R>(fr32, fr64, N + ni);
    }
    for (uint32_t k = threadIdx.x; k < P; k += blockDim.x) {
        const int64_t i = ni;
        const uint32_t kk = nk;
        const R fx = nfx, fy = nfy;
        if (k + blockDim.x < P) {
            ni = tile_point(tr, k + blockDim.x);
            nk = key[ni];
            nfx = frac_of<R>(fr32, fr64, ni);
            nfy = frac_of<R>(fr32, fr64, N + ni);
        }
        const int lx = (int)(kk % (uint32_t)Ex) - x0, ly = (int)(kk / (uint32_t)Ex) - y0;
        R wx[M2], wy[M2];
        taps<R, M2>(wp, fx, rm, rb, rw, wx);
        taps<R, M2>(wp, fy, rm, rb, rw, wy);
        for (int f = 0; f < nfield; ++f) {
            const R *lf = L + f * PT2 + ly * PT + lx;
            double acc = 0.0;
#pragma unroll
            for (int bb = 0; bb < M2; ++bb) {
                R rs = (R)0;
#pragma unroll
                for (int a = 0; a < M2; ++a) rs += wx[a] * lf[bb * PT + a];
                acc += (double)wy[bb] * (double)rs;
            }
            far[(int64_t)f * farstride + i] = acc;
        }
    }
}

// Values in binned order: val[c][k] = w_k q[perm_k][c] (w = NULL: 1), in the working
// precision and in FP64.  Grid-stride, SV_U elements per thread per trip with all
// their index and value loads issued before the first store (the value loads are
// gathers through perm); with part != NULL each block also writes the sum of its
// component-0 values, in a fixed order.  VEC: NC = 2 values of a point read as one
// 16-byte load (q 16-byte aligned).
constexpr int SV_NT = 256, SV_U = 4, SV_MAXB = 1024;

template <typename R, int NC, bool VEC>
__global__ void __launch_bounds__(SV_NT) k_set_values(const double *__restrict__ q, const double *__restrict__ w,
                                                      const uint32_t *__restrict__ perm, int64_t n,
                                                      R *__restrict__ val, double *__restrict__ val64,
                                                      double *__restrict__ part)
{
    const int64_t stride = (int64_t)gridDim.x * SV_NT;
    double acc = 0.0;
    for (int64_t k0 = blockIdx.x * (int64_t)SV_NT + threadIdx.x; k0 < n; k0 += SV_U * stride) {
        uint32_t pi[SV_U];
        double wk[SV_U], v0[SV_U], v1[SV_U];
#pragma unroll
        for (int u = 0; u < SV_U; ++u) {
            const int64_t k = k0 + u * stride;
            pi[u] = k < n ? perm[k] : 0u;
            wk[u] = (w && k < n) ? w[k] : 1.0;
        }
#pragma unroll
        for (int u = 0; u < SV_U; ++u) {
            v0[u] = v1[u] = 0.0;
            if (k0 + u * stride < n) {
                if (NC == 2 && VEC) {
                    const double2 t = reinterpret_cast<const double2 *>(q)[pi[u]];
                    v0[u] = t.x;
                    v1[u] = t.y;
                } else {
                    v0[u] = q[(int64_t)pi[u] * NC];
                    if (NC == 2) v1[u] = q[(int64_t)pi[u] * NC + 1];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < SV_U; ++u) {
            const int64_t k = k0 + u * stride;
            if (k < n) {
                const double a = wk[u] * v0[u];
                val[k] = (R)a;
                val64[k] = a;
                acc += a;
                if (NC == 2) {
                    const double b = wk[u] * v1[u];
                    val[n + k] = (R)b;
                    val64[n + k] = b;
                }
            }
        }
    }
    if (part) {
        __shared__ double sh[SV_NT];
        sh[threadIdx.x] = acc;
        __syncthreads();
        for (int h = SV_NT / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
    }
}

constexpr int SUMB = 256;
__global__ void __launch_bounds__(SUMB) k_sum_partial(const double *__restrict__ x, int64_t n,
                                                      double *__restrict__ part)
{
    __shared__ double sh[SUMB];
    double v = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)SUMB + threadIdx.x; i < n; i += (int64_t)gridDim.x * SUMB) v += x[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = SUMB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// k_spread_cells<M2, NG, TL> when a group holds at most 144 register sums (else NULL, and
// the variant is not instantiated)
using SpreadCellsKernel = void (*)(const float *, const float *, int64_t, const uint32_t *, int, int, int, int,
                                   double *, const WinPoly);
template <int M2, int NG, int TL>
SpreadCellsKernel spread_cells_kernel()
{
    if constexpr (2 * ((M2 / 2 + NG - 1) / NG) * M2 <= 144) return k_spread_cells<M2, NG, TL>;
    else return nullptr;
}

template <typename R, int M2, int TL>
hipError_t spread_t(const Plan &P, const Geom &g, int set, const Buffers &b, const void *val, int nfield,
                    double *ptile, hipStream_t st)
{
    constexpr int PT = TL + M2 - 1;
    const int ntx = (g.ext[0] + TL - 1) / TL, nty = (g.ext[1] + TL - 1) / TL;
    const int ntiles = ntx * nty;
    const size_t lds = (size_t)SPREAD_WAVES * nfield * PT * PT * sizeof(double);
    const int64_t N = set_size(g, set);
#if FN_SPREAD_CELLS
    if (std::is_same<R, float>::value) {
        // row groups of the register footprint (at most 144 sums per group)
        const int ng = P.spread_ng ? P.spread_ng : spread_default_groups(M2 / 2);
        const SpreadCellsKernel kc = ng == 1 ? spread_cells_kernel<M2, 1, TL>()
                                             : (ng == 2 ? spread_cells_kernel<M2, 2, TL>()
                                                        : (ng == 3 ? spread_cells_kernel<M2, 3, TL>() : nullptr));
        if (!kc) return hipErrorInvalidValue;
        const size_t lds1 = (size_t)SPREAD_WAVES * PT * PT * sizeof(double);
        hipError_t e = hipFuncSetAttribute((const void *)kc, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds1);
        if (e != hipSuccess) return e;
        kc<<<ntiles * nfield, SPREAD_NT, lds1, st>>>(b.fr32[set], (const float *)val, N, b.cstart[set], g.ext[0],
                                                     g.ext[1], ntx, nty, ptile, P.wpoly);
        return hipGetLastError();
    }
#endif
    auto kern = k_spread<R, M2, TL>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    kern<<<ntiles, SPREAD_NT, lds, st>>>(b.key[set], b.fr32[set], b.fr64[set], (const R *)val, N,
                                         b.cstart[set], g.ext[0], g.ext[1], ntx, nty, P.kb_b,
                                         P.win_norm, nfield, ptile, P.wpoly);
    return hipGetLastError();
}

template <typename R, int M2, int TL>
hipError_t gather_t(const Plan &P, const Geom &g, int set, const Buffers &b, const void *grid, int nfield,
                    int64_t fstride, double *far, int64_t farstride, hipStream_t st)
{
    constexpr int PT = TL + M2 - 1;
    const int ntx = (g.ext[0] + TL - 1) / TL, nty = (g.ext[1] + TL - 1) / TL;
    const int ntiles = ntx * nty;
    const size_t lds = (size_t)nfield * PT * PT * sizeof(R);
    const int64_t N = set_size(g, set);
    k_gather<R, M2, TL><<<ntiles, 256, lds, st>>>(b.key[set], b.fr32[set], b.fr64[set], N, b.cstart[set], g.ext[0],
                                                 g.ext[1], ntx, P.kb_b, P.win_norm, (const R *)grid,
                                                 fstride, nfield, far, farstride, P.wpoly);
    return hipGetLastError();
}

template <typename R, int TL>
hipError_t spread_mt(const Plan &P, const Geom &g, int set, const Buffers &b, const void *val, int nfield,
                     double *ptile, hipStream_t st)
{
    switch (P.m) {
    case 2: return spread_t<R, 4, TL>(P, g, set, b, val, nfield, ptile, st);
    case 3: return spread_t<R, 6, TL>(P, g, set, b, val, nfield, ptile, st);
    case 4: return spread_t<R, 8, TL>(P, g, set, b, val, nfield, ptile, st);
    case 5: return spread_t<R, 10, TL>(P, g, set, b, val, nfield, ptile, st);
    case 6: return spread_t<R, 12, TL>(P, g, set, b, val, nfield, ptile, st);
    case 7: return spread_t<R, 14, TL>(P, g, set, b, val, nfield, ptile, st);
    case 8: return spread_t<R, 16, TL>(P, g, set, b, val, nfield, ptile, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t spread_m(const Plan &P, const Geom &g, int set, const Buffers &b, const void *val, int nfield,
                    double *ptile, hipStream_t st)
{
    if (P.tile == 16) return spread_mt<R, 16>(P, g, set, b, val, nfield, ptile, st);
    if (P.tile == 32) return spread_mt<R, 32>(P, g, set, b, val, nfield, ptile, st);
    return hipErrorInvalidValue;
}

template <typename R, int TL>
hipError_t gather_mt(const Plan &P, const Geom &g, int set, const Buffers &b, const void *grid, int nfield,
                     int64_t fstride, double *far, int64_t farstride, hipStream_t st)
{
    switch (P.m) {
    case 2: return gather_t<R, 4, TL>(P, g, set, b, grid, nfield, fstride, far, farstride, st);
    case 3: return gather_t<R, 6, TL>(P, g, set, b, grid, nfield, fstride, far, farstride, st);
    case 4: return gather_t<R, 8, TL>(P, g, set, b, grid, nfield, fstride, far, farstride, st);
    case 5: return gather_t<R, 10, TL>(P, g, set, b, grid, nfield, fstride, far, farstride, st);
    case 6: return gather_t<R, 12, TL>(P, g, set, b, grid, nfield, fstride, far, farstride, st);
    case 7: return gather_t<R, 14, TL>(P, g, set, b, grid, nfield, fstride, far, farstride, st);
    case 8: return gather_t<R, 16, TL>(P, g, set, b, grid, nfield, fstride, far, farstride, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t gather_m(const Plan &P, const Geom &g, int set, const Buffers &b, const void *grid, int nfield, int64_t fstride,
                    double *far, int64_t farstride, hipStream_t st)
{
    if (P.tile == 16) return gather_mt<R, 16>(P, g, set, b, grid, nfield, fstride, far, farstride, st);
    if (P.tile == 32) return gather_mt<R, 32>(P, g, set, b, grid, nfield, fstride, far, farstride, st);
    return hipErrorInvalidValue;
}

}  // namespace

// Spread nfield value arrays of point set `set` into the padded tiles at ptile
// (field f of the set at ptile + f * ntiles * PT^2).
hipError_t launch_spread(int precision, const Plan &P, const Geom &g, int set, const Buffers &b, const void *val,
                         int nfield, double *ptile, hipStream_t st)
{
    return precision == FN_FP64 ? spread_m<double>(P, g, set, b, val, nfield, ptile, st)
                                : spread_m<float>(P, g, set, b, val, nfield, ptile, st);
}

hipError_t launch_fold(int precision, const Geom &g, int m, int tile, const double *ptile, int nfield, void *grid,
                       int64_t fstride, hipStream_t st)
{
    const int64_t tot = (int64_t)g.ext[0] * g.ext[1];
    const int nb = (int)((tot + 255) / 256);
    const int PT = tile + 2 * m - 1;
    const int ntx = (g.ext[0] + tile - 1) / tile, nty = (g.ext[1] + tile - 1) / tile;
    if (precision == FN_FP64)
        k_fold<double><<<nb, 256, 0, st>>>(ptile, g.ext[0], g.ext[1], ntx, nty, tile, PT, nfield,
                                           (double *)grid, fstride);
    else
        k_fold<float><<<nb, 256, 0, st>>>(ptile, g.ext[0], g.ext[1], ntx, nty, tile, PT, nfield,
                                          (float *)grid, fstride);
    return hipGetLastError();
}

// Interpolate nfield grids (grid, grid + fstride, ...) at the points of `set`.
hipError_t launch_gather(int precision, const Plan &P, const Geom &g, int set, const Buffers &b, const void *grid,
                         int nfield, int64_t fstride, double *far, int64_t farstride, hipStream_t st)
{
    return precision == FN_FP64 ? gather_m<double>(P, g, set, b, grid, nfield, fstride, far, farstride, st)
                                : gather_m<float>(P, g, set, b, grid, nfield, fstride, far, farstride, st);
}

template <typename R>
static void set_values_t(const double *q, const double *w, const uint32_t *perm, int64_t n, int ncomp, R *val,
                         double *val64, double *part, int nb, hipStream_t st)
{
    if (ncomp == 1)
        k_set_values<R, 1, false><<<nb, SV_NT, 0, st>>>(q, w, perm, n, val, val64, part);
    else if ((reinterpret_cast<uintptr_t>(q) & 15) == 0)
        k_set_values<R, 2, true><<<nb, SV_NT, 0, st>>>(q, w, perm, n, val, val64, part);
    else
        k_set_values<R, 2, false><<<nb, SV_NT, 0, st>>>(q, w, perm, n, val, val64, part);
}

hipError_t launch_set_values(const double *q, const double *w, const uint32_t *perm, int64_t n, int ncomp,
                             int precision, void *val, double *val64, double *part, int *nblk, hipStream_t st)
{
    if (nblk) *nblk = 0;
    if (n == 0) return hipSuccess;
    if (ncomp != 1 && ncomp != 2) return hipErrorInvalidValue;
    const int nb = (int)std::min<int64_t>(SV_MAXB, (n + (int64_t)SV_NT * SV_U - 1) / ((int64_t)SV_NT * SV_U));
    if (precision == FN_FP64)
        set_values_t<double>(q, w, perm, n, ncomp, (double *)val, val64, part, nb, st);
    else
        set_values_t<float>(q, w, perm, n, ncomp, (float *)val, val64, part, nb, st);
    if (nblk) *nblk = nb;
    return hipGetLastError();
}

// red[0] = sum of the np block sums (fixed order)
hipError_t launch_sum_partials(const double *part, int64_t np, double *red, hipStream_t st)
{
    k_sum_partial<<<1, SUMB, 0, st>>>(part, np, red);
    return hipGetLastError();
}

// red[0] = sum of x (fixed-order tree; red needs 1 + 256 doubles)
hipError_t launch_sum(const double *x, int64_t n, double *red, hipStream_t st)
{
    k_sum_partial<<<256, SUMB, 0, st>>>(x, n, red + 1);
    k_sum_partial<<<1, SUMB, 0, st>>>(red + 1, 256, red);
    return hipGetLastError();
}

__global__ void k_fill(double *x, int64_t n, double v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

hipError_t launch_fill(double *x, int64_t n, double v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_fill<<<(int)((n + 255) / 256), 256, 0, st>>>(x, n, v);
    return hipGetLastError();
}

}  // namespace fn
