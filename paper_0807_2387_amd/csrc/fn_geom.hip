// Geometry set-up: bounding box, torus map, binning by grid cell (stable LSD
// radix sort), sorted per-point copies and the cell-start table.
//
// Torus map: c = bounding-box midpoint, D = 2 max |r - c|, s = (1/2 - eps_B)/D,
// so every pairwise distance is at most 1/2 - eps_B on the unit torus and the
// periodized kernel never wraps.  With the centred grid coordinate v = s (r - c) G
// the point sits at grid position u = v + G/2; its window taps are
// floor(u) - m + 1 + a, a = 0..2m-1, and its "base cell" (the first tap, relative
// to the data window origin) is its bin key.  Positions are kept as (base cell,
// in-cell fraction v - floor(v)) so that differences of nearby points are exact
// to the last bit of the fraction.
#include "fn_internal.h"

#include <algorithm>
#include <cfloat>
#include <cstdlib>
#include <cstring>

namespace fn {

namespace {

constexpr int RB = 256;  // reduction block

template <int OP>  // 0 bbox (min x, min y, -max x, -max y) ; 1 max dist^2 ; 2 non-finite count
__global__ void __launch_bounds__(RB) k_reduce(const double *__restrict__ p, int64_t n, double cx,
                                               double cy, double *__restrict__ part)
{
    __shared__ double sh[4][RB];
    double v[4];
    if (OP == 0) { v[0] = v[1] = v[2] = v[3] = DBL_MAX; }
    else { v[0] = v[1] = v[2] = v[3] = 0.0; }
    for (int64_t i = blockIdx.x * (int64_t)RB + threadIdx.x; i < n; i += (int64_t)gridDim.x * RB) {
        if (OP == 0) {
            double x = p[2 * i], y = p[2 * i + 1];
            v[0] = fmin(v[0], x); v[1] = fmin(v[1], y);
            v[2] = fmin(v[2], -x); v[3] = fmin(v[3], -y);
            // NaN propagates as "not finite" through the separate check
        } else if (OP == 1) {
            double dx = p[2 * i] - cx, dy = p[2 * i + 1] - cy;
            v[0] = fmax(v[0], dx * dx + dy * dy);
        } else {
            double x = p[i];
            v[0] += (isfinite(x) ? 0.0 : 1.0);
        }
    }
    for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = RB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int k = 0; k < 4; ++k) {
                double a = sh[k][threadIdx.x], b = sh[k][threadIdx.x + s];
                sh[k][threadIdx.x] = OP == 0 ? fmin(a, b) : (OP == 1 ? fmax(a, b) : a + b);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) part[4 * blockIdx.x + k] = sh[k][0];
}

// Centred grid coordinate v = s (r - c) G (exactly t G for the torus coordinate t,
// G being a power of two); the point's taps are floor(v) + G/2 - m + 1 + a.
__global__ void k_prepare(const double *__restrict__ xy, int64_t n, double cx, double cy, double s,
                          double G, int m, int wlox, int wloy, int extx, int exty,
                          uint32_t *__restrict__ key, uint32_t *__restrict__ idx)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double vx = (s * (xy[2 * i] - cx)) * G;
    const double vy = (s * (xy[2 * i + 1] - cy)) * G;
    const int half = (int)(0.5 * G);
    int bx = (int)floor(vx) + half - m + 1 - wlox;
    int by = (int)floor(vy) + half - m + 1 - wloy;
    // the window is sized with a margin; clamping only guards against a rounding slip
    bx = min(max(bx, 0), extx - 2 * m);
    by = min(max(by, 0), exty - 2 * m);
    // x slice of the cell: the in-cell fraction vx - floor(vx) (k_finish_points forms it the
    // same way) times NEAR_SUB, exact for a power of two
    const int sub = min((int)((vx - floor(vx)) * NEAR_SUB), NEAR_SUB - 1);
    key[i] = ((uint32_t)by * (uint32_t)extx + (uint32_t)bx) * NEAR_SUB + (uint32_t)sub;
    idx[i] = (uint32_t)i;
}

// In-cell fractions v - floor(v) (exact in FP64), sorted order.
__global__ void k_finish_points(const double *__restrict__ xy, const double *__restrict__ w, int64_t n,
                                const uint32_t *__restrict__ perm, double cx, double cy, double s,
                                double G, float *__restrict__ fr32, double *__restrict__ fr64,
                                double *__restrict__ wsorted)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t i = perm[k];
    const double vx = (s * (xy[2 * (int64_t)i] - cx)) * G;
    const double vy = (s * (xy[2 * (int64_t)i + 1] - cy)) * G;
    const double fx = vx - floor(vx), fy = vy - floor(vy);
    fr32[k] = (float)fx;
    fr32[n + k] = (float)fy;
    fr64[k] = fx;
    fr64[n + k] = fy;
    if (wsorted) wsorted[k] = w[i];
}

// cstart[c] = first sorted index whose key >= c, for c in [0, ncell]
__global__ void k_cellstart(const uint32_t *__restrict__ key, int64_t n, int64_t ncell,
                            uint32_t *__restrict__ cstart)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c > ncell) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)key[mid] < c) lo = mid + 1; else hi = mid;
    }
    cstart[c] = (uint32_t)lo;
}

// csub[f] = first sorted index whose slice key >= f, for f in [0, ncell NEAR_SUB], and
// cstart[c] = csub[c NEAR_SUB]
__global__ void k_cellstart_sub(const uint32_t *__restrict__ key, int64_t n, int64_t nsub,
                                uint32_t *__restrict__ cstart, uint32_t *__restrict__ csub)
{
    int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (f > nsub) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)key[mid] < f) lo = mid + 1; else hi = mid;
    }
    csub[f] = (uint32_t)lo;
    if ((f & (NEAR_SUB - 1)) == 0) cstart[f >> NEAR_SUB_LOG2] = (uint32_t)lo;
}

__global__ void k_key_to_cell(uint32_t *__restrict__ key, int64_t n)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) key[i] >>= NEAR_SUB_LOG2;
}

// ---------------- stable LSD radix sort, 8-bit digits ----------------
constexpr int SB = 256;           // threads per sort block
constexpr int SROUNDS = 16;       // rounds of SB keys per block
constexpr int SCHUNK = SB * SROUNDS;

__global__ void __launch_bounds__(SB) k_hist(const uint32_t *__restrict__ key, int64_t n, int shift,
                                            uint32_t *__restrict__ hist, int nblk)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * SCHUNK;
    for (int r = 0; r < SROUNDS; ++r) {
        int64_t i = base + r * SB + threadIdx.x;
        if (i < n) atomicAdd(&h[(key[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of hist (256 * nblk entries) in place; one block of 1024 threads
__global__ void __launch_bounds__(1024) k_scan_hist(uint32_t *__restrict__ hist, int64_t total)
{
    __shared__ uint32_t part[1024];
    int64_t per = (total + 1023) / 1024;
    int64_t b = threadIdx.x * per, e = min(total, b + per);
    uint32_t sum = 0;
    for (int64_t i = b; i < e; ++i) sum += hist[i];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - sum;
    for (int64_t i = b; i < e; ++i) {
        uint32_t v = hist[i];
        hist[i] = run;
        run += v;
    }
}

__global__ void __launch_bounds__(SB) k_scatter(const uint32_t *__restrict__ key,
                                               const uint32_t *__restrict__ val, int64_t n, int shift,
                                               const uint32_t *__restrict__ hist, int nblk,
                                               uint32_t *__restrict__ key2, uint32_t *__restrict__ val2)
{
    __shared__ uint32_t goff[256];
    __shared__ uint32_t cnt[SB / 64][256];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    goff[tid] = hist[(int64_t)tid * nblk + blockIdx.x];
    for (int w = 0; w < SB / 64; ++w) cnt[w][tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SCHUNK;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int r = 0; r < SROUNDS; ++r) {
        int64_t i = base + r * SB + tid;
        bool valid = i < n;
        uint32_t k = valid ? key[i] : 0u;
        uint32_t v = valid ? val[i] : 0u;
        uint32_t d = (k >> shift) & 255u;
        uint64_t peers = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            uint64_t bb = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        int rank = __popcll(peers & lt);
        if (valid && rank == 0) cnt[wv][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = goff[d] + (uint32_t)rank;
            for (int w = 0; w < wv; ++w) off += cnt[w][d];
            key2[off] = k;
            val2[off] = v;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < SB / 64; ++w) { add += cnt[w][tid]; cnt[w][tid] = 0; }
        goff[tid] += add;
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_bbox(const double *p, int64_t n, double *part, int nblk, hipStream_t st)
{
    k_reduce<0><<<nblk, RB, 0, st>>>(p, n, 0.0, 0.0, part);
    return hipGetLastError();
}

hipError_t launch_maxdist(const double *p, int64_t n, double cx, double cy, double *part, int nblk,
                          hipStream_t st)
{
    k_reduce<1><<<nblk, RB, 0, st>>>(p, n, cx, cy, part);
    return hipGetLastError();
}

hipError_t launch_nonfinite(const double *p, int64_t n, double *part, int nblk, hipStream_t st)
{
    k_reduce<2><<<nblk, RB, 0, st>>>(p, n, 0.0, 0.0, part);
    return hipGetLastError();
}

hipError_t launch_prepare(const double *xy, int64_t n, double cx, double cy, double s, int G, int m,
                          int wlox, int wloy, int extx, int exty, uint32_t *key, uint32_t *idx,
                          hipStream_t st)
{
    if (n == 0) return hipSuccess;
    int nb = (int)((n + 255) / 256);
    k_prepare<<<nb, 256, 0, st>>>(xy, n, cx, cy, s, (double)G, m, wlox, wloy, extx, exty, key, idx);
    return hipGetLastError();
}

hipError_t radix_sort(uint32_t *key, uint32_t *val, uint32_t *key2, uint32_t *val2, uint32_t *hist,
                      int64_t n, int keybits, hipStream_t st)
{
    if (n <= 1) return hipSuccess;
    int nblk = (int)((n + SCHUNK - 1) / SCHUNK);
    int passes = (keybits + 7) / 8;
    if (passes % 2) passes += 1;  // even pass count leaves the result in key/val
    uint32_t *ka = key, *va = val, *kb = key2, *vb = val2;
    for (int ps = 0; ps < passes; ++ps) {
        int shift = 8 * ps;
        if (shift >= 32) shift = 24;  // an extra pass on the top digit is a stable no-op reorder
        k_hist<<<nblk, SB, 0, st>>>(ka, n, shift, hist, nblk);
        k_scan_hist<<<1, 1024, 0, st>>>(hist, (int64_t)256 * nblk);
        k_scatter<<<nblk, SB, 0, st>>>(ka, va, n, shift, hist, nblk, kb, vb);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    return hipGetLastError();
}

hipError_t launch_finish_points(const double *xy, const double *w, int64_t n, const uint32_t *perm,
                                double cx, double cy, double s, int G, float *fr32, double *fr64,
                                double *wsorted, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    int nb = (int)((n + 255) / 256);
    k_finish_points<<<nb, 256, 0, st>>>(xy, w, n, perm, cx, cy, s, (double)G, fr32, fr64, wsorted);
    return hipGetLastError();
}

__global__ void k_zero_u32(uint32_t *__restrict__ p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k_check_bins(const uint32_t *__restrict__ key, const uint32_t *__restrict__ perm,
                             const uint32_t *__restrict__ cstart, const float *__restrict__ fr32,
                             const double *__restrict__ fr64, int64_t n, int64_t ncell, uint32_t *__restrict__ cnt,
                             uint32_t *__restrict__ bad)
{
    uint32_t v = 0;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t kk = key[k];
        if ((int64_t)kk >= ncell) ++v;
        else if ((int64_t)cstart[kk] > k || (int64_t)cstart[kk + 1] <= k) ++v;
        if (k + 1 < n && key[k + 1] < kk) ++v;
        for (int d = 0; d < 2; ++d) {
            const double f = fr64[d * n + k];
            const float g = fr32[d * n + k];
            if (!(f >= 0.0 && f < 1.0)) ++v;
            if (!(g >= 0.0f && g <= 1.0f)) ++v;
        }
        const uint32_t i = perm[k];
        if ((int64_t)i >= n) ++v;
        else atomicAdd(&cnt[i], 1u);
    }
    if (v) atomicAdd(bad, v);
}

__global__ void k_check_perm(const uint32_t *__restrict__ cnt, int64_t n, uint32_t *__restrict__ bad)
{
    uint32_t v = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v += cnt[i] != 1u ? 1u : 0u;
    if (v) atomicAdd(bad, v);
}

hipError_t launch_check_bins(const uint32_t *key, const uint32_t *perm, const uint32_t *cstart, const float *fr32,
                             const double *fr64, int64_t n, int64_t ncell, uint32_t *cnt, uint32_t *bad,
                             hipStream_t st)
{
    const int nb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256));
    k_zero_u32<<<nb, 256, 0, st>>>(cnt, n);
    k_zero_u32<<<1, 64, 0, st>>>(bad, 1);
    if (n > 0) {
        k_check_bins<<<nb, 256, 0, st>>>(key, perm, cstart, fr32, fr64, n, ncell, cnt, bad);
        k_check_perm<<<nb, 256, 0, st>>>(cnt, n, bad);
    }
    return hipGetLastError();
}

bool debug_checks_from_env()
{
    const char *e = std::getenv("FEMNFFT_DEBUG_CHECKS");
    return e && *e && std::strcmp(e, "0") != 0;
}

hipError_t launch_cellstart(const uint32_t *key, int64_t n, int64_t ncell, uint32_t *cstart,
                            hipStream_t st)
{
    int nb = (int)((ncell + 1 + 255) / 256);
    k_cellstart<<<nb, 256, 0, st>>>(key, n, ncell, cstart);
    return hipGetLastError();
}

hipError_t launch_cellstart_sub(uint32_t *key, int64_t n, int64_t ncell, uint32_t *cstart, uint32_t *csub,
                                hipStream_t st)
{
    const int64_t nsub = ncell * NEAR_SUB;
    k_cellstart_sub<<<(int)((nsub + 1 + 255) / 256), 256, 0, st>>>(key, n, nsub, cstart, csub);
    if (n > 0) k_key_to_cell<<<(int)((n + 255) / 256), 256, 0, st>>>(key, n);
    return hipGetLastError();
}

}  // namespace fn
