// Near-field correction and final FP64 reduction.
//
// The far field uses the smoothed kernel K_R, which equals K(r) = -(1/2pi) ln r
// for r >= eps_I and the even polynomial T_I(r) = sum_k a_k (r/eps_I)^{2k}
// inside (matching K and its first p-1 derivatives at eps_I) -- the paper's
// "correction in the smoothing zone".  For every pair closer than eps_I this
// kernel adds s_j (K - T_I)(r) to phi and -s_j grad(K - T_I) to H; a coincident
// pair adds -s_j T_I(0) (the far field holds K_R(0) = a_0 for it; the exact sum
// has no self term).  The correction and its first p-1 derivatives vanish at
// eps_I, so pairs on the boundary of the zone contribute nothing either way.
//
// Coordinates are FP64 grid units u = (s (r - c) + 1/2) G; since G is a power
// of two, differences convert to torus units exactly.  In grid units with
// d = u_i - u_j, r2 = |d|^2, e2 = (eps_I G)^2, rho2 = r2/e2:
//   (K - T_I)(r)           = ln(G)/(2pi) - ln(r2)/(4pi) - T(rho2)
//   -grad_y (K - T_I)      = G * (1/(2 pi r2) + 2 T'(rho2)/e2) * d
// with T(x) = sum_k a_k x^k, T'(x) = sum_{k>=1} k a_k x^{k-1}.
//
// Final: phi = far + near + (ln s / 2pi) sum_j s_j,  H = s (far + near), written
// to the caller's order.  The adjoint kernels loop over targets near each source
// and produce u_j = w_j s (far + near) for H^T and u_j = w_j (far + near +
// (ln s / 2pi) sum_i v_i) for phi^T.
//
// One thread per (cell-sorted) output point; the neighbour candidates are the
// point sets' cells within rnear cells in each direction, read through the
// cell-start table, so any point density works.
#include "fn_internal.h"

namespace fn {

namespace {

constexpr double INV_2PI = 0.15915494309189533576888376337251436;
constexpr double INV_4PI = 0.07957747154594766788444188168625718;

struct NearK {
    double a[MAXP];
    int p;
};

__device__ __forceinline__ void poly2(const NearK &k, double x, double &T, double &dT)
{
    double t = k.a[k.p - 1], d = 0.0;
    for (int i = k.p - 1; i >= 1; --i) {
        d = d * x + (double)i * k.a[i];
        t = t * x + k.a[i - 1];
    }
    T = t;
    dT = d;
}

__global__ void __launch_bounds__(256) k_near_fwd(int64_t nt, const uint32_t *__restrict__ tkey,
                                                  const double *__restrict__ tu, const uint32_t *__restrict__ tperm,
                                                  int64_t ns, const double *__restrict__ su,
                                                  const double *__restrict__ sval,
                                                  const uint32_t *__restrict__ scstart, int Ex, int Ey,
                                                  const double *__restrict__ far, int64_t farstride, NearArgs na,
                                                  const double *__restrict__ sum_s, int want_phi, int want_h,
                                                  double *__restrict__ phi, double *__restrict__ H)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= nt) return;
    NearK kk;
    kk.p = na.p;
#pragma unroll
    for (int i = 0; i < MAXP; ++i) kk.a[i] = na.a[i];
    const uint32_t key = tkey[k];
    const int cx = (int)(key % (uint32_t)Ex), cy = (int)(key / (uint32_t)Ex);
    const double ux = tu[k], uy = tu[nt + k];
    const double inv_e2 = 1.0 / na.eps2g;
    const double c0 = log(1.0 / na.ginv) * INV_2PI;
    double pn = 0.0, hx = 0.0, hy = 0.0;
    const int R = na.rnear;
    const int ylo = max(cy - R, 0), yhi = min(cy + R, Ey - 1);
    const int xlo = max(cx - R, 0), xhi = min(cx + R, Ex - 1);
    for (int row = ylo; row <= yhi; ++row) {
        const int64_t rb = (int64_t)row * Ex;
        const uint32_t j0 = scstart[rb + xlo], j1 = scstart[rb + xhi + 1];
        for (uint32_t j = j0; j < j1; ++j) {
            const double dx = ux - su[j], dy = uy - su[ns + j];
            const double r2 = dx * dx + dy * dy;
            if (r2 >= na.eps2g) continue;
            const double s = sval[j];
            if (r2 == 0.0) {
                pn -= s * kk.a[0];
                continue;
            }
            double T, dT;
            poly2(kk, r2 * inv_e2, T, dT);
            if (want_phi) pn += s * (c0 - INV_4PI * log(r2) - T);
            if (want_h) {
                const double f = s * (INV_2PI / r2 + 2.0 * dT * inv_e2);
                hx += f * dx;
                hy += f * dy;
            }
        }
    }
    const int64_t i = tperm[k];
    if (want_phi) phi[i] = far[k] + pn + na.offset * sum_s[0];
    if (want_h) {
        const double G = 1.0 / na.ginv;
        H[2 * i] = na.scale * (far[farstride + k] + G * hx);
        H[2 * i + 1] = na.scale * (far[2 * farstride + k] + G * hy);
    }
}

// kind 0: H^T (V), kind 1: phi^T (v).  Loops over targets near each source.
__global__ void __launch_bounds__(256) k_near_adj(int64_t ns, const uint32_t *__restrict__ skey,
                                                  const double *__restrict__ su, const uint32_t *__restrict__ sperm,
                                                  const double *__restrict__ sw, int64_t nt,
                                                  const double *__restrict__ tu, const double *__restrict__ tval,
                                                  const uint32_t *__restrict__ tcstart, int Ex, int Ey,
                                                  const double *__restrict__ far, NearArgs na, int kind,
                                                  const double *__restrict__ sum_v, double *__restrict__ u)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= ns) return;
    NearK kk;
    kk.p = na.p;
#pragma unroll
    for (int i = 0; i < MAXP; ++i) kk.a[i] = na.a[i];
    const uint32_t key = skey[j];
    const int cx = (int)(key % (uint32_t)Ex), cy = (int)(key / (uint32_t)Ex);
    const double ux = su[j], uy = su[ns + j];
    const double inv_e2 = 1.0 / na.eps2g;
    const double c0 = log(1.0 / na.ginv) * INV_2PI;
    double acc = 0.0;
    const int R = na.rnear;
    const int ylo = max(cy - R, 0), yhi = min(cy + R, Ey - 1);
    const int xlo = max(cx - R, 0), xhi = min(cx + R, Ex - 1);
    for (int row = ylo; row <= yhi; ++row) {
        const int64_t rb = (int64_t)row * Ex;
        const uint32_t i0 = tcstart[rb + xlo], i1 = tcstart[rb + xhi + 1];
        for (uint32_t i = i0; i < i1; ++i) {
            const double dx = tu[i] - ux, dy = tu[nt + i] - uy;  // target minus source
            const double r2 = dx * dx + dy * dy;
            if (r2 >= na.eps2g) continue;
            if (kind == 1) {
                const double v = tval[i];
                if (r2 == 0.0) {
                    acc -= v * kk.a[0];
                    continue;
                }
                double T, dT;
                poly2(kk, r2 * inv_e2, T, dT);
                acc += v * (c0 - INV_4PI * log(r2) - T);
            } else {
                if (r2 == 0.0) continue;
                double T, dT;
                poly2(kk, r2 * inv_e2, T, dT);
                const double f = INV_2PI / r2 + 2.0 * dT * inv_e2;
                acc += f * (tval[i] * dx + tval[nt + i] * dy);
            }
        }
    }
    const int64_t o = sperm[j];
    if (kind == 1) u[o] = sw[j] * (far[j] + acc + na.offset * sum_v[0]);
    else u[o] = sw[j] * na.scale * (far[j] + acc / na.ginv);
}

}  // namespace

hipError_t launch_near_fwd(const Geom &g, const Buffers &b, const NearArgs &na, const double *sum_s,
                           int want_phi, int want_h, double *phi, double *H, hipStream_t st)
{
    if (g.nt == 0) return hipSuccess;
    const int nb = (int)((g.nt + 255) / 256);
    k_near_fwd<<<nb, 256, 0, st>>>(g.nt, b.key[0], b.u64[0], b.perm[0], g.ns, b.u64[1], b.val64, b.cstart[1],
                                   g.ext[0], g.ext[1], b.far, g.nt, na, sum_s, want_phi, want_h, phi, H);
    return hipGetLastError();
}

hipError_t launch_near_adj(const Geom &g, const Buffers &b, const NearArgs &na, int kind, const double *sum_v,
                           double *u, hipStream_t st)
{
    if (g.ns == 0) return hipSuccess;
    const int nb = (int)((g.ns + 255) / 256);
    k_near_adj<<<nb, 256, 0, st>>>(g.ns, b.key[1], b.u64[1], b.perm[1], b.w, g.nt, b.u64[0], b.aval64,
                                   b.cstart[0], g.ext[0], g.ext[1], b.far, na, kind, sum_v, u);
    return hipGetLastError();
}

}  // namespace fn
