// Near-field correction and final FP64 reduction.
//
// The far field uses the smoothed kernel K_R, which equals K(r) = -(1/2pi) ln r
// for r >= eps_I and the even polynomial T_I(r) = sum_k a_k (r/eps_I)^{2k}
// inside (matching K and its first p-1 derivatives at eps_I) -- the paper's
// "correction in the smoothing zone".  For every pair closer than eps_I this
// kernel adds s_j (K - T_I)(r) to phi and -s_j grad(K - T_I) to H.  A coincident
// pair is not part of the exact sum: the far field holds K_R(0) = a_0 for it and
// the final offset its share ln(s)/2pi, so it adds -s_j (a_0 + ln(s)/2pi).
// The correction and its first p-1 derivatives vanish at eps_I, so pairs on the
// boundary of the zone contribute nothing either way.
//
// Positions are (integer grid cell, FP64 in-cell fraction); a pair's offset in
// grid units is d = (c_i - c_j) + (f_i - f_j), exact up to the rounding of the
// result itself, so even points a tiny fraction of a cell apart keep their
// relative position to full FP64 precision.  G is a power of two, so grid units
// convert to torus units exactly.  With r2 = |d|^2, e2 = (eps_I G)^2 and
// x = r2/e2 = (r/eps_I)^2, and because T_I(eps_I) = K(eps_I) and
// T_I'(eps_I) = K'(eps_I) (so dT/dx = -1/(4pi) at x = 1):
//   (K - T_I)(r)           = -(1/(4pi)) ln x - U(x),   U(x) = T(x) - K(eps_I)
//   -grad_y (K - T_I)      = (2G/e2) (1/(4pi x) + T'(x)) d
// Both terms of the first line vanish at the zone edge, so the logarithm is
// only ever needed to the absolute accuracy of the result.
//
// Final: phi = far + near + (ln s / 2pi) sum_j s_j,  H = s (far + near), written
// to the caller's order.  The transposes loop over targets near each source:
// u_j = w_j s (far + near) for H^T and u_j = w_j (far + near + (ln s / 2pi)
// sum_i v_i) for phi^T.
//
// Precision: offsets, r2, x, the in-zone test, the polynomial and all sums are
// FP64.  In the mixed-precision path ln x and 1/x come from the FP32 hardware
// log2 and reciprocal (x rounded to FP32 first): ln x is then off by ~1e-7
// absolute, (1/4pi) ln x by < 1e-8, and 1/(4pi x) by ~1e-7 of itself.
//
// Work decomposition: one workgroup per NBX x NBY block of "home" cells of the
// output point set; the points of the other set lying in the block's rows and
// columns widened by rnear cells are staged into LDS in chunks of at most CAP
// points (coalesced copies), so any point density works.  Each thread owns one
// home point at a time and, for every staged row within rnear, loops over the
// cells within the disk bound of its own cell, two staged points per trip with
// a branch-free pair body (two independent dependency chains per lane).
#include "fn_internal.h"

#include <algorithm>

namespace fn {

namespace {

constexpr double INV_4PI = 0.07957747154594766788444188168625718;
// The home block shape (bx x by cells, bx by = 256) and the staging capacity are
// run-time values (NearShape, chosen per direction by the plan or the autotuner).
// Wider than tall is the usual winner: the 64 home points of a wave (cell order) then
// mostly share one home row, so their row windows have the same vertical gaps and
// similar trip counts (measured: 16 x 16 -> 32 x 8 cut the forward near field by 7%
// and the adjoint by 9%, at 2.0 points per cell and a radius of 5 cells).
constexpr int NTH = 256;         // threads per block
constexpr int NSEG_MAX = 16;     // home row segments per block (by), at most
constexpr int MAXRN = 32;        // largest near radius in cells
constexpr int MAXROWS = NSEG_MAX + 2 * MAXRN + 2;

enum { MODE_FWD_BOTH = 0, MODE_ADJ_H = 1, MODE_ADJ_PHI = 2, MODE_COUNT = 3, MODE_FWD_PHI = 4, MODE_FWD_H = 5 };

struct NearSets {
    // output ("home") set
    int64_t n_out;
    const uint32_t *key_out;
    const double *f_out;          // [2][n_out] in-cell fractions
    const uint32_t *perm_out;
    const uint32_t *cs_out;
    const double *far;            // [3][n_out] (fwd) or [n_out] (adjoint)
    const double *w_out;          // source weights (adjoints)
    // input set
    int64_t n_in;
    const uint32_t *key_in;
    const double *f_in;           // [2][n_in] in-cell fractions
    const uint32_t *cs_in;
    const uint32_t *csub_in;      // starts of the cells' NEAR_SUB x slices [ncell NEAR_SUB + 1]
    const double *pay;            // fwd: s [n_in]; adj H: V [2][n_in]; adj phi: v [n_in]
    int Ex, Ey, nbx;
    int bx, by;                   // home block shape, cells
    uint32_t cap;                 // staging capacity, points per LDS chunk
    int accum;                    // forward only: add the near part to phi / H instead of writing far + near
    const uint32_t *blocks;       // home blocks to run (block i of the launch is blocks[i]); NULL: all
};

// U(x) = sum_{k<P} c_k x^k and U'(x) in one Horner sweep (the derivative
// accumulates the running value: synthetic division); the coefficients are
// kernel arguments, so they live in scalar registers.  lead = c[P-1] comes in a
// vector register: a VALU instruction takes one scalar operand, so a scalar
// leading coefficient would cost a register copy in every call.
template <int P, typename T>
__device__ __forceinline__ void poly2(const T *c, T lead, T x, T &u, T &du)
{
    T t = lead, d = T(0);
#pragma unroll
    for (int i = P - 2; i >= 0; --i) {
        d = (i == P - 2) ? t : fma(d, x, t);
        t = fma(t, x, c[i]);
    }
    u = t;
    du = d;
}

// U'(x) by plain Horner over its own coefficients (k+1) u_{k+1}.
template <int P>
__device__ __forceinline__ double poly_d(const double *dc, double lead, double x)
{
    if (P < 2) return 0.0;
    double t = lead;  // dc[P - 2], in a vector register
#pragma unroll
    for (int i = P - 3; i >= 0; --i) t = fma(t, x, dc[i]);
    return t;
}

// 1/x for a normal positive x: hardware estimate refined by two Newton steps
// (each step squares the relative error, from ~2^-26 to below 2^-53).
__device__ __forceinline__ double rcp64(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// ln x for a normal positive x: x = 2^e m with m in [sqrt(1/2), sqrt(2)),
// ln m = 2 atanh(f), f = (m - 1)/(m + 1), |f| <= 0.1716, by its series up to
// f^19 (truncation below 3e-16 absolute); the series coefficients 1/(2k+1) and
// ln 2 (split in two parts) come in as kernel arguments.
__device__ __forceinline__ double ln64(double x, const NearArgs &na)
{
    int e = __builtin_amdgcn_frexp_exp(x);
    double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1)
    const bool lo = m < 0.70710678118654752440;
    m = lo ? 2.0 * m : m;
    e = lo ? e - 1 : e;
    const double f = (m - 1.0) * rcp64(m + 1.0);
    const double z = f * f;
    double s = na.lc[8];
#pragma unroll
    for (int k = 7; k >= 0; --k) s = fma(s, z, na.lc[k]);
    const double f2 = f + f;
    const double lnm = fma(f2 * z, s, f2);
    const double de = (double)e;
    return fma(de, na.ln2hi, fma(de, na.ln2lo, lnm));
}

constexpr double LN2_4PI = 0.05515890334192413571;  // ln(2)/(4 pi)

// x = (r/eps_I)^2 + XMIN keeps ln x and 1/x finite (XMIN enters through the
// innermost FMA, so x costs two instructions in the mixed path).  In the mixed path this
// moves only pairs closer than ~1e-14 cells; in the FP64 path the shift is
// below any representable offset.
constexpr double XMIN32 = 1e-30;
constexpr double XMIN64 = 1e-300;

// One pair, given the FP64 offset d (home minus staged; grid units, or units of
// eps_I G cells in the mixed path, where the caller passes e2 = 1).  The zone
// test masks the accumulation (pairs with r2 >= e2 add nothing).  A coincident
// pair (r2 = 0) adds phi_X = -(ln(XMIN)/(4pi) + U(XMIN)) to phi here -- replaced
// by czero afterwards (k_coincident) -- and, since d = 0, nothing to H.  kind 0:
// phi and H with weight s; kind 1: H only; kind 2: phi only; kind 3: the
// adjoint of H, weight (V0, V1).  The H accumulators hold
// sum s (1/(4pi x) + T'(x)) d; the caller applies 2G/e2 (2G/(eps_I G) in the
// mixed path).
template <int KIND, int P, bool F32>
__device__ __forceinline__ void pair(const NearArgs &na, double lead, double e2, double dx, double dy, double w0,
                                     double w1, double &a0, double &a1, double &a2)
{
    constexpr bool PHI = KIND == 0 || KIND == 2;
    constexpr bool GRAD = KIND == 0 || KIND == 1 || KIND == 3;
    // mixed path: offsets come in units of eps_I, so x = r2 + XMIN and the zone is x < 1
    // (adding XMIN below 1e-14 cannot move x across 1); FP64 path: the zone test on r2
    const double r2 = F32 ? 0.0 : fma(dx, dx, dy * dy);
    const double x = F32 ? fma(dx, dx, fma(dy, dy, XMIN32)) : fma(r2, na.inv_e2, XMIN64);
    double u = 0.0, du = 0.0;
    if (PHI) poly2<P, double>(na.u, lead, x, u, du);
    else du = poly_d<P>(na.du, lead, x);
    double lnx = 0.0, rx = 0.0;
    if (F32) {
        const float xf = (float)x;
        if (PHI) lnx = (double)__builtin_amdgcn_logf(xf);  // log2
        if (GRAD) rx = (double)__builtin_amdgcn_rcpf(xf);
    } else {
        if (PHI) lnx = ln64(x, na);
        if (GRAD) rx = rcp64(x);
    }
    if ((F32 ? x : r2) < e2) {
        if (PHI) {
            const double phi_t = fma(F32 ? -LN2_4PI : -INV_4PI, lnx, -u);
            a0 = fma(w0, phi_t, a0);
        }
        if (GRAD) {
            const double g = fma(INV_4PI, rx, du);
            if (KIND == 3) {
                a0 = fma(g, fma(w0, dx, w1 * dy), a0);
            } else {
                const double f = w0 * g;
                a1 = fma(f, dx, a1);
                a2 = fma(f, dy, a2);
            }
        }
    }
}

__device__ __forceinline__ int find_seg(const uint32_t *pre, int nseg, uint32_t k)
{
    int lo = 0, hi = nseg - 1;  // largest s with pre[s] <= k
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= k) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Dynamic LDS of k_near: staged in-cell fractions (double2), payloads [PAY][cap] (double)
// and, in the FP64 path, cell column offsets (uint16).
inline size_t near_lds_bytes(uint32_t cap, int pay, bool f32)
{
    return (size_t)cap * (sizeof(double2) + pay * sizeof(double)) + (f32 ? 0 : (size_t)cap * sizeof(uint16_t));
}

template <int MODE, int P, bool F32>
__global__ void __launch_bounds__(NTH) k_near(NearSets S, NearArgs na, const double *__restrict__ sum_in,
                                              double *__restrict__ out0, double *__restrict__ out1)
{
    constexpr bool FWD = MODE == MODE_FWD_BOTH || MODE == MODE_FWD_PHI || MODE == MODE_FWD_H;
    constexpr bool WANT_PHI = MODE == MODE_FWD_BOTH || MODE == MODE_FWD_PHI || MODE == MODE_ADJ_PHI;
    constexpr bool WANT_H = MODE == MODE_FWD_BOTH || MODE == MODE_FWD_H;
    constexpr int PAY = MODE == MODE_ADJ_H ? 2 : 1;
    constexpr int KIND = MODE == MODE_ADJ_H ? 3 : (WANT_PHI && WANT_H ? 0 : (WANT_H ? 1 : 2));
    const uint32_t CAP = S.cap;
    extern __shared__ double2 near_lds[];
    double2 *sxy = near_lds;                                            // in-cell fractions [CAP]
    double *spay0 = reinterpret_cast<double *>(near_lds + CAP);         // payloads [PAY][CAP]
    double *spay1 = spay0 + (PAY - 1) * CAP;
    uint16_t *scx = reinterpret_cast<uint16_t *>(spay0 + PAY * CAP);    // cell column offsets (FP64 path)
    __shared__ uint32_t hpre[NSEG_MAX + 1], hstart[NSEG_MAX];  // home row segments
    __shared__ uint32_t ipre[MAXROWS + 1], istart[MAXROWS];    // input rows

    const int Ex = S.Ex, Ey = S.Ey, R = na.rnear;
    const int NBX = S.bx, NBY = S.by, NSEG = S.by;
    const int bid = S.blocks ? (int)S.blocks[blockIdx.x] : (int)blockIdx.x;
    const int bx = bid % S.nbx, by = bid / S.nbx;
    const int hx0 = bx * NBX, hy0 = by * NBY;
    const int iy0 = max(hy0 - R, 0), iy1 = min(hy0 + NBY + R, Ey);
    const int ix0 = max(hx0 - R, 0), ix1 = min(hx0 + NBX + R, Ex);
    const int nirow = iy1 - iy0;
    const int tid = threadIdx.x;

    if (tid < NSEG) {  // segment = one row of the home block
        const int y = hy0 + tid;
        const int x0 = hx0, x1 = min(x0 + NBX, Ex);
        uint32_t s0 = 0, cnt = 0;
        if (y < Ey && x0 < Ex) {
            const int64_t rb = (int64_t)y * Ex;
            s0 = S.cs_out[rb + x0];
            cnt = S.cs_out[rb + x1] - s0;
        }
        hstart[tid] = s0;
        hpre[tid + 1] = cnt;
    }
    for (int r = tid; r < nirow; r += NTH) {
        const int64_t rb = (int64_t)(iy0 + r) * Ex;
        const uint32_t s0 = S.cs_in[rb + ix0];
        istart[r] = s0;
        ipre[r + 1] = S.cs_in[rb + ix1] - s0;
    }
    __syncthreads();
    if (tid == 0) {
        hpre[0] = 0;
        for (int s = 1; s <= NSEG; ++s) hpre[s] += hpre[s - 1];
        ipre[0] = 0;
        for (int r = 1; r <= nirow; ++r) ipre[r] += ipre[r - 1];
    }
    __syncthreads();
    const uint32_t nhome = hpre[NSEG], nin = ipre[nirow];
    if (nhome == 0) return;  // uniform
    if (FWD && S.accum && nin == 0) return;  // nothing to add to this block's targets (uniform)

    const double e2 = na.eps2g;
    // leading polynomial coefficient, pinned to a vector register (see poly2)
    double lead = (KIND == 0 || KIND == 2) ? na.u[P - 1] : na.du[P < 2 ? 0 : P - 2];
    asm volatile("" : "+v"(lead));

    for (uint32_t hb = 0; hb < nhome; hb += NTH) {
        const uint32_t k = hb + tid;
        const bool valid = k < nhome;
        int64_t gi = -1;
        int cx = 0, cy = 0;
        double px = 0.0, py = 0.0;
        if (valid) {
            const int sgi = find_seg(hpre, NSEG, k);
            gi = (int64_t)hstart[sgi] + (k - hpre[sgi]);
            const uint32_t key = S.key_out[gi];
            cx = (int)(key % (uint32_t)Ex);
            cy = (int)(key / (uint32_t)Ex);
            px = S.f_out[gi];
            py = S.f_out[S.n_out + gi];
        }
        const int hcx = cx - ix0, hcy = cy - iy0;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (uint32_t c_lo = 0; c_lo < nin; c_lo += CAP) {
            const uint32_t c_hi = min(nin, c_lo + CAP);
            __syncthreads();
            for (uint32_t kk = c_lo + tid; kk < c_hi; kk += NTH) {
                const int r = find_seg(ipre, nirow, kk);
                const int64_t j = (int64_t)istart[r] + (kk - ipre[r]);
                const uint32_t kj = S.key_in[j];
                const uint32_t qcx = kj % (uint32_t)Ex - (uint32_t)ix0;
                if (F32) {
                    // block-local coordinates in units of eps_I G cells: rounded to ~1e-15,
                    // exact enough for the FP32 arithmetic of this path
                    sxy[kk - c_lo] = make_double2(((double)qcx + S.f_in[j]) * na.inv_eg,
                                                  ((double)(kj / (uint32_t)Ex - (uint32_t)iy0) + S.f_in[S.n_in + j]) * na.inv_eg);
                } else {
                    sxy[kk - c_lo] = make_double2(S.f_in[j], S.f_in[S.n_in + j]);
                    scx[kk - c_lo] = (uint16_t)qcx;
                }
                spay0[kk - c_lo] = S.pay[j];
                if (PAY == 2) spay1[kk - c_lo] = S.pay[S.n_in + j];
            }
            __syncthreads();
            if (!valid) continue;
            const int r_first = find_seg(ipre, nirow, c_lo);
            const int r_last = find_seg(ipre, nirow, c_hi - 1);
            const int ylo = max(r_first, hcy - R), yhi = min(r_last, hcy + R);
            const double hx = (double)hcx + px;
            const double hxs = hx * na.inv_eg, hys = ((double)hcy + py) * na.inv_eg;
            // raw bounds of the points of row r that can lie within eps_I: the x slices
            // (NEAR_SUB per cell, the sort's second key) meeting [hx - w, hx + w], w from the
            // vertical gap between the home point and row r (padded against rounding); an
            // empty range where the gap alone exceeds eps_I
            auto bounds = [&](int r, uint32_t &blo, uint32_t &bhi) {
                const double gap = r < hcy ? (double)(hcy - r - 1) + py : (r > hcy ? (double)(r - hcy) - py : 0.0);
                const double h2 = e2 - gap * gap;
                const double w = (double)__builtin_amdgcn_sqrtf((float)fmax(h2, 0.0)) + 1e-3;  // hardware sqrt, ~1 ulp: far inside the margin
                const int f0 = max((int)floor((hx - w) * NEAR_SUB), 0);
                const int f1 = h2 > 0.0 ? min((int)floor((hx + w) * NEAR_SUB), (ix1 - ix0) * NEAR_SUB - 1) : f0 - 1;
                const int64_t rb = ((int64_t)(iy0 + r) * Ex + ix0) * NEAR_SUB;
                blo = S.csub_in[rb + f0];
                bhi = S.csub_in[rb + f1 + 1];
            };
            uint32_t nlo = 0, nhi = 0;
            if (ylo <= yhi) bounds(ylo, nlo, nhi);
            for (int r = ylo; r <= yhi; ++r) {
                const uint32_t blo = nlo, bhi = nhi;
                if (r < yhi) bounds(r + 1, nlo, nhi);  // next row's loads overlap this row's pairs
                uint32_t lo = ipre[r] + (blo - istart[r]);
                uint32_t hi = ipre[r] + (bhi - istart[r]);
                lo = max(lo, c_lo) - c_lo;
                hi = min(hi, c_hi);
                hi = hi > c_lo ? hi - c_lo : 0;
                const double dyc = (double)(hcy - r);  // every staged point of this row is in row r
                if (MODE == MODE_COUNT) {
                    for (uint32_t jj = lo; jj < hi; ++jj) {
                        const double dx = (double)(hcx - (int)scx[jj]) + (px - sxy[jj].x);
                        const double dy = dyc + (py - sxy[jj].y);
                        a0 += fma(dx, dx, dy * dy) < e2 ? 1.0 : 0.0;
                    }
                    continue;
                }
                // home minus staged: target minus source (forward), source minus target (adjoint)
                if (F32) {
                    const double2 *pq = sxy + lo;
                    const double *pw0 = spay0 + lo;
                    const double *pw1 = spay1 + lo;
                    uint32_t n = hi > lo ? hi - lo : 0;
                    for (; n >= 2; n -= 2, pq += 2, pw0 += 2, pw1 += 2) {
                        const double2 q0 = pq[0], q1 = pq[1];
                        const double w00 = pw0[0], w10 = pw0[1];
                        const double w01 = PAY == 2 ? pw1[0] : 0.0, w11 = PAY == 2 ? pw1[1] : 0.0;
                        pair<KIND, P, F32>(na, lead, 1.0, hxs - q0.x, hys - q0.y, w00, w01, a0, a1, a2);
                        pair<KIND, P, F32>(na, lead, 1.0, hxs - q1.x, hys - q1.y, w10, w11, a0, a1, a2);
                    }
                    if (n) {
                        const double2 q0 = pq[0];
                        const double w00 = pw0[0], w01 = PAY == 2 ? pw1[0] : 0.0;
                        pair<KIND, P, F32>(na, lead, 1.0, hxs - q0.x, hys - q0.y, w00, w01, a0, a1, a2);
                    }
                    continue;
                }
                const double2 *pq = sxy + lo;
                const uint16_t *pc = scx + lo;
                const double *pw0 = spay0 + lo;
                const double *pw1 = spay1 + lo;
                uint32_t n = hi > lo ? hi - lo : 0;
                for (; n >= 2; n -= 2, pq += 2, pc += 2, pw0 += 2, pw1 += 2) {
                    const double2 q0 = pq[0], q1 = pq[1];
                    const int x0 = pc[0], x1 = pc[1];
                    const double w00 = pw0[0], w10 = pw0[1];
                    const double w01 = PAY == 2 ? pw1[0] : 0.0, w11 = PAY == 2 ? pw1[1] : 0.0;
                    pair<KIND, P, F32>(na, lead, e2, (double)(hcx - x0) + (px - q0.x), dyc + (py - q0.y), w00, w01, a0, a1, a2);
                    pair<KIND, P, F32>(na, lead, e2, (double)(hcx - x1) + (px - q1.x), dyc + (py - q1.y), w10, w11, a0, a1, a2);
                }
                if (n) {
                    const double2 q0 = pq[0];
                    const int x0 = pc[0];
                    const double w00 = pw0[0], w01 = PAY == 2 ? pw1[0] : 0.0;
                    pair<KIND, P, F32>(na, lead, e2, (double)(hcx - x0) + (px - q0.x), dyc + (py - q0.y), w00, w01, a0, a1, a2);
                }
            }
        }
        if (valid) {
            const int64_t o = S.perm_out[gi];
            const double G2 = F32 ? 2.0 * na.inv_eg / na.ginv : 2.0 / (na.ginv * na.eps2g);
            if (FWD && S.accum) {
                if (WANT_PHI) out0[o] += a0;
                if (WANT_H) {
                    out1[2 * o] = fma(na.scale * G2, a1, out1[2 * o]);
                    out1[2 * o + 1] = fma(na.scale * G2, a2, out1[2 * o + 1]);
                }
            } else if (FWD) {
                if (WANT_PHI) out0[o] = S.far[gi] + a0 + na.offset * sum_in[0];
                if (WANT_H) {
                    out1[2 * o] = na.scale * fma(G2, a1, S.far[S.n_out + gi]);
                    out1[2 * o + 1] = na.scale * fma(G2, a2, S.far[2 * S.n_out + gi]);
                }
            } else if (MODE == MODE_COUNT) {
                out0[o] = a0;
            } else if (MODE == MODE_ADJ_H) {
                // the accumulated offsets are source minus target: flip the sign
                out0[o] = S.w_out[gi] * na.scale * fma(-G2, a0, S.far[gi]);
            } else {
                out0[o] = S.w_out[gi] * (S.far[gi] + a0 + na.offset * sum_in[0]);
            }
        }
    }
}

// Coincident pairs (equal cell and fractions, i.e. r2 = 0 in the near kernel)
// received phi_X there; add (czero - phi_X) times the other set's values in the
// home point's own cell.  Forward: phi_i += (czero - phi_X) sum s_j; adjoint of
// phi: u_j += w_j (czero - phi_X) sum v_i.  Runs only when set_geometry found
// such pairs.
template <int P, bool F32>
__global__ void __launch_bounds__(256) k_coincident(NearSets S, NearArgs na, int adjoint, double *__restrict__ out)
{
    const int64_t gi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gi >= S.n_out) return;
    const uint32_t key = S.key_out[gi];
    const double px = S.f_out[gi], py = S.f_out[S.n_out + gi];
    double acc = 0.0;
    for (uint32_t j = S.cs_in[key]; j < S.cs_in[key + 1]; ++j)
        if (S.f_in[j] == px && S.f_in[S.n_in + j] == py) acc += S.pay[j];
    if (acc == 0.0) return;
    double phx = 0.0, d1 = 0.0, d2 = 0.0;
    pair<2, P, F32>(na, na.u[P - 1], F32 ? 1.0 : na.eps2g, 0.0, 0.0, 1.0, 0.0, phx, d1, d2);
    const double f = (na.czero - phx) * acc;
    const int64_t o = S.perm_out[gi];
    out[o] += adjoint ? S.w_out[gi] * f : f;
}

// Count, per home point, the points of the other set at exactly its position.
__global__ void __launch_bounds__(256) k_coincident_count(NearSets S, double *__restrict__ cnt)
{
    const int64_t gi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gi >= S.n_out) return;
    const uint32_t key = S.key_out[gi];
    const double px = S.f_out[gi], py = S.f_out[S.n_out + gi];
    double c = 0.0;
    for (uint32_t j = S.cs_in[key]; j < S.cs_in[key + 1]; ++j)
        c += (S.f_in[j] == px && S.f_in[S.n_in + j] == py) ? 1.0 : 0.0;
    cnt[gi] = c;
}

template <int MODE, int P>
hipError_t launch_p(int nblk, hipStream_t st, const NearSets &S, const NearArgs &na, const double *sum, double *o0,
                    double *o1)
{
    constexpr int PAY = MODE == MODE_ADJ_H ? 2 : 1;
    const size_t lds = near_lds_bytes(S.cap, PAY, na.f32 != 0);
    const void *k = na.f32 ? (const void *)k_near<MODE, P, true> : (const void *)k_near<MODE, P, false>;
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (na.f32)
        k_near<MODE, P, true><<<nblk, NTH, lds, st>>>(S, na, sum, o0, o1);
    else
        k_near<MODE, P, false><<<nblk, NTH, lds, st>>>(S, na, sum, o0, o1);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_mode(int nblk, hipStream_t st, const NearSets &S, const NearArgs &na, const double *sum, double *o0,
                       double *o1)
{
    switch (na.p) {
#define FN_NEAR_CASE(PP) \
    case PP: return launch_p<MODE, PP>(nblk, st, S, na, sum, o0, o1);
    FN_NEAR_CASE(1) FN_NEAR_CASE(2) FN_NEAR_CASE(3) FN_NEAR_CASE(4) FN_NEAR_CASE(5) FN_NEAR_CASE(6)
    FN_NEAR_CASE(7) FN_NEAR_CASE(8) FN_NEAR_CASE(9) FN_NEAR_CASE(10) FN_NEAR_CASE(11) FN_NEAR_CASE(12)
#undef FN_NEAR_CASE
    default: return hipErrorInvalidValue;
    }
}

// Home set out_set against input set in_set (targets against a source set, or a
// source set against the targets).  The sorted arrays of a source set start at its
// base within the source arrays; far-field results follow the home set's order.
NearSets make_sets(const Geom &g, const Buffers &b, int out_set, int in_set, const NearShape &sh)
{
    NearSets S{};
    S.n_out = set_size(g, out_set);
    S.key_out = b.key[out_set];
    S.f_out = b.fr64[out_set];
    S.perm_out = b.perm[out_set];
    S.cs_out = b.cstart[out_set];
    S.far = out_set ? b.far + set_base(g, out_set) : b.far;
    S.w_out = out_set ? b.w + set_base(g, out_set) : nullptr;
    S.n_in = set_size(g, in_set);
    S.key_in = b.key[in_set];
    S.f_in = b.fr64[in_set];
    S.cs_in = b.cstart[in_set];
    S.csub_in = b.csub[in_set];
    S.pay = out_set ? b.aval64 : b.val64 + set_base(g, in_set);
    S.Ex = g.ext[0];
    S.Ey = g.ext[1];
    S.bx = sh.bx;
    S.by = sh.by;
    S.cap = (uint32_t)sh.cap;
    S.nbx = (g.ext[0] + sh.bx - 1) / sh.bx;
    S.accum = 0;
    S.blocks = nullptr;
    return S;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v)
{
    if (threadIdx.x == 0) p[0] = v;
}

// Home blocks with work: home points in the block and, if need_in, points of the
// input set within R cells of it.  One thread per block; the list order depends on
// the atomics, the blocks' results do not.
__global__ void k_block_list(NearSets S, int nblk, int R, int need_in, uint32_t cap, uint32_t *__restrict__ list,
                             uint32_t *__restrict__ count)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblk) return;
    const int NBX = S.bx, NBY = S.by;
    const int bx = b % S.nbx, by = b / S.nbx;
    const int hx0 = bx * NBX, hy0 = by * NBY;
    const int hx1 = min(hx0 + NBX, S.Ex), hy1 = min(hy0 + NBY, S.Ey);
    uint32_t home = 0;
    for (int y = hy0; y < hy1; ++y) home += S.cs_out[(int64_t)y * S.Ex + hx1] - S.cs_out[(int64_t)y * S.Ex + hx0];
    if (home == 0) return;
    if (need_in) {
        const int iy0 = max(hy0 - R, 0), iy1 = min(hy0 + NBY + R, S.Ey);
        const int ix0 = max(hx0 - R, 0), ix1 = min(hx0 + NBX + R, S.Ex);
        uint32_t in = 0;
        for (int y = iy0; y < iy1; ++y) in += S.cs_in[(int64_t)y * S.Ex + ix1] - S.cs_in[(int64_t)y * S.Ex + ix0];
        if (in == 0) return;
    }
    const uint32_t slot = atomicAdd(count, 1u);
    if (slot < cap) list[slot] = (uint32_t)b;  // a count above cap is reported by the host
}

template <int P>
hipError_t coincident_p(const NearSets &S, const NearArgs &na, int adjoint, double *out, hipStream_t st)
{
    const int nb = (int)((S.n_out + 255) / 256);
    if (na.f32)
        k_coincident<P, true><<<nb, 256, 0, st>>>(S, na, adjoint, out);
    else
        k_coincident<P, false><<<nb, 256, 0, st>>>(S, na, adjoint, out);
    return hipGetLastError();
}

}  // namespace

// phi (forward, out_set 0 against source set in_set) or the phi adjoint (source set
// out_set against the targets): replace phi_X by czero for coincident pairs.
hipError_t launch_near_coincident(const Geom &g, const Buffers &b, const NearArgs &na, int out_set, int in_set,
                                  double *out, hipStream_t st)
{
    if (set_size(g, out_set) == 0 || set_size(g, in_set) == 0) return hipSuccess;
    NearSets S = make_sets(g, b, out_set, in_set, NearShape{});
    switch (na.p) {
#define FN_CO_CASE(PP) \
    case PP: return coincident_p<PP>(S, na, out_set != 0, out, st);
    FN_CO_CASE(1) FN_CO_CASE(2) FN_CO_CASE(3) FN_CO_CASE(4) FN_CO_CASE(5) FN_CO_CASE(6)
    FN_CO_CASE(7) FN_CO_CASE(8) FN_CO_CASE(9) FN_CO_CASE(10) FN_CO_CASE(11) FN_CO_CASE(12)
#undef FN_CO_CASE
    default: return hipErrorInvalidValue;
    }
}

// cnt [n_tgt]: points of source set in_set at exactly each (sorted) target's position
hipError_t launch_coincident_count(const Geom &g, const Buffers &b, int in_set, double *cnt, hipStream_t st)
{
    if (g.nt == 0) return hipSuccess;
    if (set_size(g, in_set) == 0) return launch_fill(cnt, g.nt, 0.0, st);
    const NearSets S = make_sets(g, b, 0, in_set, NearShape{});
    k_coincident_count<<<(int)((g.nt + 255) / 256), 256, 0, st>>>(S, cnt);
    return hipGetLastError();
}

int near_blocks(const Geom &g, const NearShape &sh)
{
    return ((g.ext[0] + sh.bx - 1) / sh.bx) * ((g.ext[1] + sh.by - 1) / sh.by);
}

bool near_shape_ok(const NearShape &sh)
{
    const bool dims = (sh.bx == 16 && sh.by == 16) || (sh.bx == 32 && sh.by == 8) || (sh.bx == 64 && sh.by == 4);
    return dims && sh.cap >= 128 && sh.cap <= 2048 && sh.cap % 64 == 0;
}

int64_t near_blocks_bound(int64_t emax)
{
    // the largest count over the allowed home block shapes
    const int dims[3][2] = {{16, 16}, {32, 8}, {64, 4}};
    int64_t best = 0;
    for (const auto &d : dims) best = std::max<int64_t>(best, ((emax + d[0] - 1) / d[0]) * ((emax + d[1] - 1) / d[1]));
    return best;
}

hipError_t launch_block_list(const Geom &g, const Buffers &b, const NearShape &sh, int out_set, int in_set, int R,
                             int need_in, uint32_t *list, uint32_t cap, uint32_t *count, hipStream_t st)
{
    const int nblk = near_blocks(g, sh);
    const NearSets S = make_sets(g, b, out_set, in_set, sh);
    k_fill_u32<<<1, 1, 0, st>>>(count, 0u);
    k_block_list<<<(nblk + 255) / 256, 256, 0, st>>>(S, nblk, R, need_in, cap, list, count);
    return hipGetLastError();
}

hipError_t launch_near_fwd(const Geom &g, const Buffers &b, const NearArgs &na, const NearShape &sh, int in_set,
                           int accum, const double *sum_s, int want_phi, int want_h, double *phi, double *H,
                           const uint32_t *blocks, int nblocks, hipStream_t st)
{
    if (g.nt == 0) return hipSuccess;
    if (!near_shape_ok(sh)) return hipErrorInvalidValue;
    NearSets S = make_sets(g, b, 0, in_set, sh);
    S.accum = accum;
    S.blocks = blocks;
    const int nblk = blocks ? nblocks : near_blocks(g, sh);
    if (nblk == 0) return hipSuccess;
    if (want_phi && want_h) return launch_mode<MODE_FWD_BOTH>(nblk, st, S, na, sum_s, phi, H);
    if (want_phi) return launch_mode<MODE_FWD_PHI>(nblk, st, S, na, sum_s, phi, H);
    return launch_mode<MODE_FWD_H>(nblk, st, S, na, sum_s, phi, H);
}

// kind 0: H^T (V), kind 1: phi^T (v), kind 2: count pairs closer than the class radius
// per source.  u is the part of the output that belongs to source set out_set.
hipError_t launch_near_adj(const Geom &g, const Buffers &b, const NearArgs &na, const NearShape &sh, int out_set,
                           int kind, const double *sum_v, double *u, const uint32_t *blocks, int nblocks,
                           hipStream_t st)
{
    if (set_size(g, out_set) == 0) return hipSuccess;
    if (!near_shape_ok(sh)) return hipErrorInvalidValue;
    NearSets S = make_sets(g, b, out_set, 0, sh);
    S.blocks = blocks;
    const int nblk = blocks ? nblocks : near_blocks(g, sh);
    if (nblk == 0) return hipSuccess;
    if (kind == 0) return launch_mode<MODE_ADJ_H>(nblk, st, S, na, sum_v, u, nullptr);
    if (kind == 1) return launch_mode<MODE_ADJ_PHI>(nblk, st, S, na, sum_v, u, nullptr);
    const size_t lds = near_lds_bytes(S.cap, 1, false);
    hipError_t e = hipFuncSetAttribute((const void *)k_near<MODE_COUNT, 1, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    k_near<MODE_COUNT, 1, false><<<nblk, NTH, lds, st>>>(S, na, sum_v, u, nullptr);
    return hipGetLastError();
}

}  // namespace fn
