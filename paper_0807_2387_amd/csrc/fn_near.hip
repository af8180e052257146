// Near-field correction and final FP64 reduction.
//
// The far field uses the smoothed kernel K_R, which equals K(r) = -(1/2pi) ln r
// for r >= eps_I and the even polynomial T_I(r) = sum_k a_k (r/eps_I)^{2k}
// inside (matching K and its first p-1 derivatives at eps_I) -- the paper's
// "correction in the smoothing zone".  For every pair closer than eps_I this
// kernel adds s_j (K - T_I)(r) to phi and -s_j grad(K - T_I) to H.  A coincident
// pair is not part of the exact sum: the far field holds K_R(0) = a_0 for it and
// the final offset its share ln(s)/2pi, so it adds -s_j (a_0 + ln(s)/2pi).  The correction and its first p-1 derivatives vanish at
// eps_I, so pairs on the boundary of the zone contribute nothing either way.
//
// Positions are (integer grid cell, FP64 in-cell fraction); a pair's offset in
// grid units is d = (c_i - c_j) + (f_i - f_j), exact up to the rounding of the
// result itself, so even points a tiny fraction of a cell apart keep their
// relative position to full FP64 precision.  G is a power of two, so grid units
// convert to torus units exactly.  In grid units, with r2 = |d|^2,
// e2 = (eps_I G)^2, rho2 = r2/e2:
//   (K - T_I)(r)           = ln(G)/(2pi) - ln(r2)/(4pi) - T(rho2)
//   -grad_y (K - T_I)      = G * (1/(2 pi r2) + 2 T'(rho2)/e2) * d
// with T(x) = sum_k a_k x^k, T'(x) = sum_{k>=1} k a_k x^{k-1}.
//
// Final: phi = far + near + (ln s / 2pi) sum_j s_j,  H = s (far + near), written
// to the caller's order.  The transposes loop over targets near each source:
// u_j = w_j s (far + near) for H^T and u_j = w_j (far + near + (ln s / 2pi)
// sum_i v_i) for phi^T.
//
// Work decomposition: one workgroup per NB x NB block of "home" cells of the
// output point set.  The points of the other set lying in the block's rows and
// columns widened by rnear cells are staged into LDS in chunks of at most CAP
// points (coalesced copies), so any point density works.  Each thread owns up
// to TPT home points and, for every staged row, loops only over the cells that
// can hold a point within eps_I of its own cell.  Everything is FP64.
#include "fn_internal.h"

namespace fn {

namespace {

constexpr double INV_2PI = 0.15915494309189533576888376337251436;
constexpr double INV_4PI = 0.07957747154594766788444188168625718;
constexpr int NB = 16;           // home block edge, cells
constexpr int NTH = 256;         // threads per block
constexpr int TPT = 1;           // home points per thread per batch
constexpr int MAXROWS = NB + 2 * 64 + 2;

enum { MODE_FWD = 0, MODE_ADJ_H = 1, MODE_ADJ_PHI = 2 };

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
    const double *pay;            // fwd: s [n_in]; adj H: V [2][n_in]; adj phi: v [n_in]
    int Ex, Ey, nbx;
};

// T(x) = sum_{k<P} a_k x^k and T'(x) = sum_{k>=1} k a_k x^{k-1}, Horner, unrolled; the
// coefficients are kernel arguments, so they live in scalar registers.
template <int P>
__device__ __forceinline__ void poly2(const NearArgs &na, double x, double &T, double &dT)
{
    double t = na.a[P - 1], d = 0.0;
#pragma unroll
    for (int i = P - 1; i >= 1; --i) {
        d = fma(d, x, na.da[i]);
        t = fma(t, x, na.a[i - 1]);
    }
    T = t;
    dT = d;
}

template <int P>
__device__ __forceinline__ double poly_d(const NearArgs &na, double x)
{
    double d = 0.0;
#pragma unroll
    for (int i = P - 1; i >= 1; --i) d = fma(d, x, na.da[i]);
    return d;
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
// ln m = 2 atanh(f), f = (m - 1)/(m + 1), |f| <= 0.1716, by its series to the
// f^21 term (truncation below 1e-18 relative); ln 2 is split in two parts.
__device__ __forceinline__ double ln64(double x)
{
    int e = __builtin_amdgcn_frexp_exp(x);
    double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double f = (m - 1.0) * rcp64(m + 1.0);
    const double z = f * f;
    double s = 1.0 / 21.0;
    s = fma(s, z, 1.0 / 19.0);
    s = fma(s, z, 1.0 / 17.0);
    s = fma(s, z, 1.0 / 15.0);
    s = fma(s, z, 1.0 / 13.0);
    s = fma(s, z, 1.0 / 11.0);
    s = fma(s, z, 1.0 / 9.0);
    s = fma(s, z, 1.0 / 7.0);
    s = fma(s, z, 1.0 / 5.0);
    s = fma(s, z, 1.0 / 3.0);
    const double lnm = fma(2.0 * f * z, s, 2.0 * f);
    const double de = (double)e;
    return fma(de, 0.693147180559945286227, fma(de, 2.319046813846299558e-17, lnm));
}

__device__ __forceinline__ int find_row(const uint32_t *pre, int nrow, uint32_t k)
{
    int lo = 0, hi = nrow - 1;  // largest r with pre[r] <= k
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= k) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int MODE, int CAP, int P>
__global__ void __launch_bounds__(NTH) k_near(NearSets S, NearArgs na, const double *__restrict__ sum_in,
                                              int want_phi, int want_h, double *__restrict__ out0,
                                              double *__restrict__ out1)
{
    constexpr int PAY = MODE == MODE_ADJ_H ? 2 : 1;
    __shared__ double2 sxy[CAP];     // in-cell fractions
    __shared__ uint32_t scell[CAP];  // cell offsets from the region origin, x | y << 16
    __shared__ double spay[PAY][CAP];
    __shared__ uint32_t hpre[NB + 1], hstart[NB];          // home rows
    __shared__ uint32_t ipre[MAXROWS + 1], istart[MAXROWS]; // input rows

    const int Ex = S.Ex, Ey = S.Ey, R = na.rnear;
    const int bx = blockIdx.x % S.nbx, by = blockIdx.x / S.nbx;
    const int hx0 = bx * NB, hy0 = by * NB;
    const int hx1 = min(hx0 + NB, Ex);
    const int nhrow = min(NB, Ey - hy0);
    const int iy0 = max(hy0 - R, 0), iy1 = min(hy0 + NB + R, Ey);
    const int ix0 = max(hx0 - R, 0), ix1 = min(hx0 + NB + R, Ex);
    const int nirow = iy1 - iy0;
    const int tid = threadIdx.x;

    if (tid < nhrow) {
        const int64_t rb = (int64_t)(hy0 + tid) * Ex;
        const uint32_t s0 = S.cs_out[rb + hx0];
        hstart[tid] = s0;
        hpre[tid + 1] = S.cs_out[rb + hx1] - s0;
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
        for (int r = 1; r <= nhrow; ++r) hpre[r] += hpre[r - 1];
        ipre[0] = 0;
        for (int r = 1; r <= nirow; ++r) ipre[r] += ipre[r - 1];
    }
    __syncthreads();
    const uint32_t nhome = hpre[nhrow], nin = ipre[nirow];
    if (nhome == 0) return;  // uniform

    const double e2 = na.eps2g, inv_e2 = 1.0 / na.eps2g;
    const double c0 = log(1.0 / na.ginv) * INV_2PI;

    for (uint32_t hb = 0; hb < nhome; hb += NTH * TPT) {
        double px[TPT], py[TPT], acc0[TPT], acc1[TPT], acc2[TPT];  // px, py: home fractions
        int cx[TPT], cy[TPT];
        int64_t gi[TPT];
#pragma unroll
        for (int t = 0; t < TPT; ++t) {
            const uint32_t k = hb + tid + t * NTH;
            acc0[t] = acc1[t] = acc2[t] = 0.0;
            gi[t] = -1;
            cx[t] = cy[t] = 0;
            px[t] = py[t] = 0.0;
            if (k < nhome) {
                const int r = find_row(hpre, nhrow, k);
                const int64_t i = (int64_t)hstart[r] + (k - hpre[r]);
                gi[t] = i;
                const uint32_t key = S.key_out[i];
                cx[t] = (int)(key % (uint32_t)Ex);
                cy[t] = (int)(key / (uint32_t)Ex);
                px[t] = S.f_out[i];
                py[t] = S.f_out[S.n_out + i];
            }
        }
        for (uint32_t c_lo = 0; c_lo < nin; c_lo += CAP) {
            const uint32_t c_hi = min(nin, c_lo + (uint32_t)CAP);
            __syncthreads();
            for (uint32_t k = c_lo + tid; k < c_hi; k += NTH) {
                const int r = find_row(ipre, nirow, k);
                const int64_t j = (int64_t)istart[r] + (k - ipre[r]);
                sxy[k - c_lo] = make_double2(S.f_in[j], S.f_in[S.n_in + j]);
                const uint32_t kj = S.key_in[j];
                scell[k - c_lo] = (kj % (uint32_t)Ex - (uint32_t)ix0) | ((kj / (uint32_t)Ex - (uint32_t)iy0) << 16);
                spay[0][k - c_lo] = S.pay[j];
                if (PAY == 2) spay[PAY - 1][k - c_lo] = S.pay[S.n_in + j];
            }
            __syncthreads();
            const int r_first = find_row(ipre, nirow, c_lo);
            const int r_last = find_row(ipre, nirow, c_hi - 1);
#pragma unroll
            for (int t = 0; t < TPT; ++t) {
                if (gi[t] < 0) continue;
                const int ylo = max(r_first, cy[t] - R - iy0), yhi = min(r_last, cy[t] + R - iy0);
                for (int r = ylo; r <= yhi; ++r) {
                    const int ady = abs(iy0 + r - cy[t]);
                    const double a = (double)max(ady - 1, 0);
                    const int xr = min(R, (int)(sqrt(max(e2 - a * a, 0.0)) + 1.0));
                    const int c0c = max(cx[t] - xr, ix0), c1c = min(cx[t] + xr, ix1 - 1);
                    if (c0c > c1c) continue;
                    const int64_t rb = (int64_t)(iy0 + r) * Ex;
                    uint32_t lo = ipre[r] + (S.cs_in[rb + c0c] - istart[r]);
                    uint32_t hi = ipre[r] + (S.cs_in[rb + c1c + 1] - istart[r]);
                    lo = max(lo, c_lo) - c_lo;
                    hi = min(hi, c_hi);
                    hi = hi > c_lo ? hi - c_lo : 0;
                    const double tx = px[t], ty = py[t];
                    const int hcx = cx[t] - ix0, hcy = cy[t] - iy0;
                    double a0 = acc0[t], a1 = acc1[t], a2 = acc2[t];
                    for (uint32_t jj = lo; jj < hi; ++jj) {
                        const double2 q = sxy[jj];
                        const uint32_t pc = scell[jj];
                        const int qcx = (int)(pc & 0xffffu), qcy = (int)(pc >> 16);
                        // fwd: target minus source; adjoint: target (input) minus source (home)
                        const double dx = MODE == MODE_FWD ? (double)(hcx - qcx) + (tx - q.x)
                                                           : (double)(qcx - hcx) + (q.x - tx);
                        const double dy = MODE == MODE_FWD ? (double)(hcy - qcy) + (ty - q.y)
                                                           : (double)(qcy - hcy) + (q.y - ty);
                        const double r2 = fma(dx, dx, dy * dy);
                        if (r2 >= e2) continue;
                        if (MODE == MODE_ADJ_H) {
                            if (r2 == 0.0) continue;
                            const double dT = poly_d<P>(na, r2 * inv_e2);
                            const double f = fma(2.0 * dT, inv_e2, INV_2PI * rcp64(r2));
                            a0 = fma(f, fma(spay[0][jj], dx, spay[1][jj] * dy), a0);
                        } else {
                            const double s = spay[0][jj];
                            if (r2 == 0.0) {
                                a0 = fma(-s, na.a[0] + na.offset, a0);
                                continue;
                            }
                            double T, dT;
                            poly2<P>(na, r2 * inv_e2, T, dT);
                            if (MODE == MODE_ADJ_PHI || want_phi) a0 = fma(s, c0 - INV_4PI * ln64(r2) - T, a0);
                            if (MODE == MODE_FWD && want_h) {
                                const double f = s * fma(2.0 * dT, inv_e2, INV_2PI * rcp64(r2));
                                a1 = fma(f, dx, a1);
                                a2 = fma(f, dy, a2);
                            }
                        }
                    }
                    acc0[t] = a0;
                    acc1[t] = a1;
                    acc2[t] = a2;
                }
            }
        }
#pragma unroll
        for (int t = 0; t < TPT; ++t) {
            const int64_t i = gi[t];
            if (i < 0) continue;
            const int64_t o = S.perm_out[i];
            if (MODE == MODE_FWD) {
                if (want_phi) out0[o] = S.far[i] + acc0[t] + na.offset * sum_in[0];
                if (want_h) {
                    const double G = 1.0 / na.ginv;
                    out1[2 * o] = na.scale * fma(G, acc1[t], S.far[S.n_out + i]);
                    out1[2 * o + 1] = na.scale * fma(G, acc2[t], S.far[2 * S.n_out + i]);
                }
            } else if (MODE == MODE_ADJ_H) {
                out0[o] = S.w_out[i] * na.scale * fma(1.0 / na.ginv, acc0[t], S.far[i]);
            } else {
                out0[o] = S.w_out[i] * (S.far[i] + acc0[t] + na.offset * sum_in[0]);
            }
        }
    }
}

constexpr int CAP_FWD = 2048;
constexpr int CAP_ADJ = 2048;

template <int MODE, int CAP, int P>
hipError_t launch_p(int nblk, hipStream_t st, const NearSets &S, const NearArgs &na, const double *sum,
                    int want_phi, int want_h, double *o0, double *o1)
{
    k_near<MODE, CAP, P><<<nblk, NTH, 0, st>>>(S, na, sum, want_phi, want_h, o0, o1);
    return hipGetLastError();
}

template <int MODE, int CAP>
hipError_t launch_mode(int nblk, hipStream_t st, const NearSets &S, const NearArgs &na, const double *sum,
                       int want_phi, int want_h, double *o0, double *o1)
{
    switch (na.p) {
#define FN_NEAR_CASE(PP) \
    case PP: return launch_p<MODE, CAP, PP>(nblk, st, S, na, sum, want_phi, want_h, o0, o1);
    FN_NEAR_CASE(1) FN_NEAR_CASE(2) FN_NEAR_CASE(3) FN_NEAR_CASE(4) FN_NEAR_CASE(5) FN_NEAR_CASE(6)
    FN_NEAR_CASE(7) FN_NEAR_CASE(8) FN_NEAR_CASE(9) FN_NEAR_CASE(10) FN_NEAR_CASE(11) FN_NEAR_CASE(12)
#undef FN_NEAR_CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_near_fwd(const Geom &g, const Buffers &b, const NearArgs &na, const double *sum_s,
                           int want_phi, int want_h, double *phi, double *H, hipStream_t st)
{
    if (g.nt == 0) return hipSuccess;
    NearSets S{};
    S.n_out = g.nt;
    S.key_out = b.key[0];
    S.f_out = b.fr64[0];
    S.perm_out = b.perm[0];
    S.cs_out = b.cstart[0];
    S.far = b.far;
    S.w_out = nullptr;
    S.n_in = g.ns;
    S.key_in = b.key[1];
    S.f_in = b.fr64[1];
    S.cs_in = b.cstart[1];
    S.pay = b.val64;
    S.Ex = g.ext[0];
    S.Ey = g.ext[1];
    S.nbx = (g.ext[0] + NB - 1) / NB;
    const int nby = (g.ext[1] + NB - 1) / NB;
    return launch_mode<MODE_FWD, CAP_FWD>(S.nbx * nby, st, S, na, sum_s, want_phi, want_h, phi, H);
}

hipError_t launch_near_adj(const Geom &g, const Buffers &b, const NearArgs &na, int kind, const double *sum_v,
                           double *u, hipStream_t st)
{
    if (g.ns == 0) return hipSuccess;
    NearSets S{};
    S.n_out = g.ns;
    S.key_out = b.key[1];
    S.f_out = b.fr64[1];
    S.perm_out = b.perm[1];
    S.cs_out = b.cstart[1];
    S.far = b.far;
    S.w_out = b.w;
    S.n_in = g.nt;
    S.key_in = b.key[0];
    S.f_in = b.fr64[0];
    S.cs_in = b.cstart[0];
    S.pay = b.aval64;
    S.Ex = g.ext[0];
    S.Ey = g.ext[1];
    S.nbx = (g.ext[0] + NB - 1) / NB;
    const int nby = (g.ext[1] + NB - 1) / NB;
    if (kind == 0) return launch_mode<MODE_ADJ_H, CAP_ADJ>(S.nbx * nby, st, S, na, sum_v, 0, 0, u, nullptr);
    return launch_mode<MODE_ADJ_PHI, CAP_ADJ>(S.nbx * nby, st, S, na, sum_v, 0, 0, u, nullptr);
}

}  // namespace fn
