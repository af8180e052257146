// The fast summation in 3D: the discrete Green sum of the paper's eq. (2) with the 3D
// Green function given with eq. (1), G(r) = 1/(4 pi r), its field H = -grad phi and the
// transpose of the H map, by the NFFT method of the paper's "NFFT" section (a grid of
// about p^3 N points in 3D), FP64 throughout.
//
// Steps (the 2D path's, in three dimensions):
//   torus map   c = bounding-box midpoint, D = 2 max |p - c|, s = (1/2 - eps_B)/D; for mapped
//               points t = s (r - c), G(y - x) = s K(|t_y - t_x|), K(r) = 1/(4 pi r), so
//               phi = s (torus sum) and H = s^2 (torus gradient sum)
//   plan        K_R = T_I (even polynomial of degree 2p-2 matching K and p-1 derivatives at
//               eps_I) inside eps_I, K up to 1/2 - eps_B, T_B to 1/2, constant beyond;
//               b_l = DFT of K_R on the n^3 grid (bandwidth n: G/2, or any even n up to
//               3G/4), by separable cosine sums since b_l is real and even;
//               W_l = omega_l b_l / prod_d psihat(l_d/G)^2
//   spread      g_k = sum_j s_j prod_d psi(G t_jd - k_d), (2m)^3 taps from per-point tap
//               tables: each tile of ST^3 cells accumulates its footprint in LDS (each
//               value updated by one wave in point order, no atomics), and a fold adds the
//               overlapping footprints per grid point in tile order
//   FFT         G^3 complex, Stockham line transforms through LDS along each axis
//   multiply    W_l, and -2 pi i l_d W_l for the field; phi with H_z and H_x with H_y share
//               one complex inverse transform each (real fields A + iB)
//   gather      per target over the (2m)^3 taps of the four real grids
//   near field  per target over the cells within eps_I: s_j (K - T_I)(r) and
//               -s_j grad(K - T_I); a pair at distance 0 adds -s_j a_0 (the far field holds
//               K_R(0) = a_0 for it, the exact sum leaves it out)
//   adjoint     V spread at the targets (3 fields, the first two as one complex grid),
//               sum_d 2 pi i l_d W_l F_d, inverse transform, gather at the sources,
//               transposed near field; u = w s^2 (..)
#include "fn_fft_dev.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace fn3 {

using fn::FFT_EPT;
using fn::MAXM;
using fn::MAXP;

constexpr double PI = 3.14159265358979323846264338327950288;
constexpr double INV_4PI = 0.07957747154594766788444188168625718;
constexpr int MAXG3 = 256;
constexpr int NT = 256;

struct Plan3 {
    int G = 0, n = 0, m = 0, p = 0, log2G = 0;
    double eps_I = 0, eps_B = 0, kb_b = 0, i0mb = 0;
    double a[MAXP] = {0};
    std::vector<double> cB, psihat;
    std::vector<double> twG;   // pass-ordered twiddles of G-point lines (staged_twiddles)
    std::vector<double> ctab;  // cos(2 pi k / n), k < n: the plan's cosine sums
};

struct Geom3 {
    int64_t nt = 0, ns = 0;
    double c[3] = {0, 0, 0};
    double s = 0;
    int wlo[3] = {0, 0, 0}, ext[3] = {0, 0, 0};
    int rnear = 0;
    int64_t near_pairs = 0;
};

struct Buf3 {
    double *W = nullptr;              // [(n/2+1)^3]
    double2 *twG = nullptr;
    double *ctab = nullptr;
    uint32_t *key[2] = {nullptr, nullptr}, *perm[2] = {nullptr, nullptr}, *cstart[2] = {nullptr, nullptr};
    double4 *pos[2] = {nullptr, nullptr}; // [N] positions in grid units (base cell + fraction)
    double *taps[2] = {nullptr, nullptr}; // [N][3][2m] window taps
    double *w = nullptr;              // sorted source weights
    double *val = nullptr;            // s_j sorted
    double *aval = nullptr;           // adjoint input V [3][nt] sorted
    double2 *grid[3] = {nullptr, nullptr, nullptr};  // G^3 complex
    double *far = nullptr;            // [4][max(nt, ns)]
    double *red = nullptr;            // reduction scratch
    double *tiles = nullptr;          // spread tile footprints [tile][F^3]
    uint32_t *skey = nullptr, *sval = nullptr, *hist = nullptr;
};

}  // namespace fn3

struct fn3_ctx {
    fn_params prm{};
    fn3::Plan3 plan;
    fn3::Geom3 geom;
    fn3::Buf3 buf;
    hipStream_t stream = nullptr;
    int device = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool plan_ready = false, geom_ready = false, charges_ready = false;
    uint64_t geom_gen = 0;  // successful fn3_set_geometry calls
    bool debug_checks = false;  // FEMNFFT_DEBUG_CHECKS: validate the binning after fn3_set_geometry
    std::string err;
    // stage timing (fn3_set_profiling): event pairs recorded on the stream around each stage
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;
    std::vector<int> prof_stage;
    size_t prof_next = 0;
    fn_profile prof{};
};

namespace fn3 {

static thread_local std::string g_err3;

// ------------------------------------------------------------------ host plan

static double bessel_i0(double x)
{
    const double q = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 300; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

// r^q K^{(q)}(r) for K = 1/(4 pi r)
static double K_scaled_deriv(int q, double r)
{
    double f = 1.0;
    for (int i = 2; i <= q; ++i) f *= i;
    return ((q % 2) ? -1.0 : 1.0) * f / (4.0 * PI * r);
}

static double falling(int a, int q)
{
    if (q > a) return 0.0;
    double r = 1.0;
    for (int i = 0; i < q; ++i) r *= (double)(a - i);
    return r;
}

static bool solve(std::vector<double> A, std::vector<double> b, int n, std::vector<double> &x)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0.0) return false;
        if (piv != c) {
            for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < n; ++r) {
            const double f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    x.assign(n, 0.0);
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * x[k];
        x[r] = s / A[r * n + r];
    }
    return true;
}


static bool build_plan(const fn_params &prm, Plan3 &P, std::string &err)
{
    P.G = prm.grid;
    P.n = prm.n ? prm.n : prm.grid / 2;
    P.m = prm.m;
    P.p = prm.p;
    P.eps_I = prm.eps_I;
    P.eps_B = prm.eps_B;
    while ((1 << P.log2G) < P.G) ++P.log2G;
    P.kb_b = PI * (2.0 - (double)P.n / P.G);
    P.i0mb = bessel_i0(P.m * P.kb_b);
    {
        const int p = P.p;
        std::vector<double> A(p * p), b(p), x;
        for (int q = 0; q < p; ++q) {
            for (int k = 0; k < p; ++k) A[q * p + k] = falling(2 * k, q);
            b[q] = K_scaled_deriv(q, P.eps_I);
        }
        if (!solve(A, b, p, x)) { err = "inner regularization system is singular"; return false; }
        for (int k = 0; k < MAXP; ++k) P.a[k] = k < p ? x[k] : 0.0;
    }
    {
        const int p = P.p;
        const double rB = 0.5 - P.eps_B;
        P.cB.assign(2 * p - 1, 0.0);
        double fact = 1.0;
        for (int q = 0; q < p; ++q) {
            if (q > 0) fact *= q;
            P.cB[q] = K_scaled_deriv(q, rB) * std::pow(P.eps_B / rB, q) / fact;
        }
        if (p > 1) {
            const int nu = p - 1;
            std::vector<double> A(nu * nu), b(nu), x;
            for (int qi = 0; qi < nu; ++qi) {
                const int q = qi + 1;
                double rhs = 0.0;
                for (int k = 0; k < p; ++k) rhs -= P.cB[k] * falling(k, q);
                b[qi] = rhs;
                for (int ki = 0; ki < nu; ++ki) A[qi * nu + ki] = falling(p + ki, q);
            }
            if (!solve(A, b, nu, x)) { err = "boundary regularization system is singular"; return false; }
            for (int ki = 0; ki < nu; ++ki) P.cB[p + ki] = x[ki];
        }
    }
    P.psihat.resize(P.n / 2 + 1);
    for (int l = 0; l <= P.n / 2; ++l) {
        const double w = 2.0 * PI * l / P.G;
        P.psihat[l] = bessel_i0(P.m * std::sqrt(P.kb_b * P.kb_b - w * w)) / P.i0mb;
    }
    fn::staged_twiddles(P.G, P.twG);  // pass-ordered table of the G-point lines
    P.ctab.resize(P.n);
    for (int k = 0; k < P.n; ++k) P.ctab[k] = (double)std::cos(2.0L * (long double)PI * k / P.n);
    return true;
}

// ------------------------------------------------------------------ device helpers

// Kaiser-Bessel window at t cells, sinh(b z)/(pi z I0(m b)) with z = sqrt(m^2 - t^2), evaluated
// as (e^{-b t^2/(z+m)} - e^{-b(z+m)}) wnorm / z, wnorm = 1/(2 pi I0(m b) e^{-m b}) (the same
// value: e^{b(z-m)} = e^{-b t^2/(z+m)}); zero for |t| >= m.
__device__ __forceinline__ double kb_psi(double t, double m, double b, double wnorm)
{
    const double t2 = t * t;
    const double z2 = m * m - t2;
    if (!(z2 > 0.0)) return 0.0;
    const double z = sqrt(z2);
    const double zm = z + m;
    return (exp(-b * t2 / zm) - exp(-b * zm)) * wnorm / z;
}


// ------------------------------------------------------------------ geometry kernels

// per block: min x, y, z and max x, y, z (as negated mins), and a non-finite count
__global__ void k3_bbox(const double *__restrict__ p, int64_t n, double *__restrict__ part)
{
    __shared__ double sh[7][NT];
    double v[7] = {1e308, 1e308, 1e308, 1e308, 1e308, 1e308, 0.0};
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        for (int d = 0; d < 3; ++d) {
            const double x = p[3 * i + d];
            if (!isfinite(x)) { v[6] += 1.0; continue; }
            v[d] = fmin(v[d], x);
            v[3 + d] = fmin(v[3 + d], -x);
        }
    for (int k = 0; k < 7; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 7; ++k)
                sh[k][threadIdx.x] = k < 6 ? fmin(sh[k][threadIdx.x], sh[k][threadIdx.x + h])
                                           : sh[k][threadIdx.x] + sh[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 7) part[7 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k3_maxdist(const double *__restrict__ p, int64_t n, double cx, double cy, double cz,
                           double *__restrict__ part)
{
    __shared__ double sh[NT];
    double v = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const double a = p[3 * i] - cx, b = p[3 * i + 1] - cy, c = p[3 * i + 2] - cz;
        v = fmax(v, a * a + b * b + c * c);
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k3_nonfinite(const double *__restrict__ w, int64_t n, double *__restrict__ part)
{
    __shared__ double sh[NT];
    double v = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        v += isfinite(w[i]) ? 0.0 : 1.0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

struct Map3 {
    double c[3], s, G;
    int m, wlo[3], ext[3];
};

// key = base (first tap) cell in the data window, x fastest; idx = i
__global__ void k3_prepare(const double *__restrict__ p, int64_t n, Map3 mp, uint32_t *__restrict__ key,
                           uint32_t *__restrict__ idx)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int half = (int)(0.5 * mp.G);
    int b[3];
    for (int d = 0; d < 3; ++d) {
        const double v = (mp.s * (p[3 * i + d] - mp.c[d])) * mp.G;
        b[d] = (int)floor(v) + half - mp.m + 1 - mp.wlo[d];
        b[d] = min(max(b[d], 0), mp.ext[d] - 2 * mp.m);  // guards a rounding slip only
    }
    key[i] = ((uint32_t)b[2] * (uint32_t)mp.ext[1] + (uint32_t)b[1]) * (uint32_t)mp.ext[0] + (uint32_t)b[0];
    idx[i] = (uint32_t)i;
}

// sorted positions (grid units from the data window origin: base cell + in-cell fraction per
// axis, w unused), window taps [n][3][2m] and sorted weights
__global__ void k3_finish(const double *__restrict__ p, const double *__restrict__ w, int64_t n,
                          const uint32_t *__restrict__ perm, Map3 mp, double kb_b, double wnorm,
                          double4 *__restrict__ pos, double *__restrict__ taps, double *__restrict__ wsorted)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t i = perm[k];
    const int M2 = 2 * mp.m;
    const int half = (int)(0.5 * mp.G);
    double q[3];
    for (int d = 0; d < 3; ++d) {
        const double v = (mp.s * (p[3 * (int64_t)i + d] - mp.c[d])) * mp.G;
        const double fl = floor(v);
        const double f = v - fl;
        q[d] = (fl + (double)(half - mp.m + 1 - mp.wlo[d])) + f;
        for (int a = 0; a < M2; ++a) taps[(k * 3 + d) * M2 + a] = kb_psi(f + (double)(mp.m - 1 - a), mp.m, kb_b, wnorm);
    }
    pos[k] = make_double4(q[0], q[1], q[2], 0.0);
    if (wsorted) wsorted[k] = w[i];
}

// ------------------------------------------------------------------ plan kernels

// b_l = (1/n^3) sum_{j in I_n^3} K_R(|j|/n) e^{-2 pi i j.l/n} is real and even in every
// component of j and l (K_R is radial and the grid I_n = {-n/2 + 1, ..., n/2} is symmetric
// up to its Nyquist index, where e^{-2 pi i j l/n} is real), so it is a separable cosine
// sum over the half grid j_d in [0, n/2] with weight 1 at j_d = 0 and n/2 and 2 between:
//   b_l = (1/n^3) sum_j prod_d (om_{j_d} cos(2 pi j_d l_d / n)) K_R(|j|/n),  l_d in [0, n/2].
// Three passes of (n/2 + 1)-term sums (any even n: oversampling 2 or 4/3 alike).
// Samples on the half grid: a[(j2 nh1 + j1) nh1 + j0] = K_R(|j|/n).
__global__ void k3_kr_samples(double *__restrict__ a, int n, const double *__restrict__ coef, int p,
                              double eps_I, double eps_B, const double *__restrict__ cB, int ncB)
{
    const int nh1 = n / 2 + 1;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nh1 * nh1 * nh1) return;
    const int j0 = (int)(idx % nh1), j1 = (int)((idx / nh1) % nh1), j2 = (int)(idx / ((int64_t)nh1 * nh1));
    const double r = sqrt((double)j0 * j0 + (double)j1 * j1 + (double)j2 * j2) / n;
    const double rB = 0.5 - eps_B;
    double v;
    if (r < eps_I) {
        const double rho2 = (r / eps_I) * (r / eps_I);
        double acc = 0.0;
        for (int k = p - 1; k >= 0; --k) acc = acc * rho2 + coef[k];
        v = acc;
    } else if (r <= rB) {
        v = INV_4PI / r;
    } else {
        const double t = r > 0.5 ? 1.0 : (r - rB) / eps_B;
        double acc = 0.0;
        for (int k = ncB - 1; k >= 0; --k) acc = acc * t + cB[k];
        v = acc;
    }
    a[idx] = v;
}

// One axis of the cosine sums: out[.., l, ..] = sum_j om_j cos(2 pi j l / n) in[.., j, ..] along
// `axis` (0: the fastest index), over the (n/2 + 1)^3 half grid; ctab[k] = cos(2 pi k / n).
__global__ void k3_cos_pass(const double *__restrict__ in, double *__restrict__ out, int n, int axis,
                            const double *__restrict__ ctab)
{
    const int nh = n / 2, nh1 = nh + 1;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nh1 * nh1 * nh1) return;
    const int64_t stride = axis == 0 ? 1 : (axis == 1 ? nh1 : (int64_t)nh1 * nh1);
    const int l = (int)((idx / stride) % nh1);
    const double *line = in + (idx - (int64_t)l * stride);
    double acc = 0.0;
    int jl = 0;  // (j l) mod n
    for (int j = 0; j <= nh; ++j) {
        const double om = (j == 0 || j == nh) ? 1.0 : 2.0;
        acc = fma(om * ctab[jl], line[(int64_t)j * stride], acc);
        jl += l;
        if (jl >= n) jl -= n;
    }
    out[idx] = acc;
}

// W[(l0 (nh+1) + l1)(nh+1) + l2] = omega(l) b_l / prod psihat(l_d)^2 for l_d in [0, n/2];
// bl holds n^3 b_l on the half grid (b_l is symmetric in its three components)
__global__ void k3_make_W(const double *__restrict__ bl, int n, const double *__restrict__ psihat,
                          double *__restrict__ W)
{
    const int nh = n / 2, nh1 = nh + 1;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nh1 * nh1 * nh1) return;
    const int l0 = (int)(idx / ((int64_t)nh1 * nh1)), l1 = (int)((idx / nh1) % nh1), l2 = (int)(idx % nh1);
    const double b = bl[idx] / ((double)n * n * n);
    const double om = (l0 == nh ? 0.5 : 1.0) * (l1 == nh ? 0.5 : 1.0) * (l2 == nh ? 0.5 : 1.0);
    const double ph = psihat[l0] * psihat[l1] * psihat[l2];
    W[idx] = om * b / (ph * ph);
}

// ------------------------------------------------------------------ FFT passes

// A set of indices along one axis of the G grid: an interval [lo, lo + len) (the data
// window), the band {0..nh} U {G-nh..G-1} (the frequencies the multiplier keeps), or all.
struct Set3 {
    int kind;  // 0 interval, 1 band, 2 all
    int lo, len;
};

__device__ __forceinline__ int set_count(const Set3 &s, int N, int nh)
{
    return s.kind == 0 ? s.len : (s.kind == 1 ? 2 * nh + 1 : N);
}
__device__ __forceinline__ int set_at(const Set3 &s, int i, int N, int nh)
{
    return s.kind == 0 ? s.lo + i : (s.kind == 1 ? (i <= nh ? i : N - 2 * nh - 1 + i) : i);
}
__device__ __forceinline__ bool set_has(const Set3 &s, int e, int N, int nh)
{
    return s.kind == 0 ? (unsigned)(e - s.lo) < (unsigned)s.len : (s.kind == 1 ? (e <= nh || e >= N - nh) : true);
}

// One pass of line transforms along `axis` of an N^3 complex cube (x fastest), in place:
// the lines are those whose other two coordinates lie in su (the faster of the two axes)
// x sv; elements outside `ld` are read as zero, and only elements in `stv` are written
// back.  Forward C2C; inverse as conj(FFT(conj(.))).  A block holds PER lines (one set of
// NT = N/FFT_EPT threads each) with consecutive su coordinates, so for axes 1 and 2 the
// PER lines' elements at one position are adjacent in memory and the copies coalesce.
__global__ void __launch_bounds__(512) k3_pass(double2 *__restrict__ a, int N, int log2N, int axis, int inv, int nh,
                                               Set3 su, Set3 sv, Set3 ld, Set3 stv, const double2 *__restrict__ tw)
{
    using namespace fn::fftd;
    extern __shared__ double2 sh3[];
    const int NT = N / FFT_EPT, PER = blockDim.x / NT;
    const int cu = set_count(su, N, nh);
    const int iv = blockIdx.y;
    const int iu0 = blockIdx.x * PER;
    const int v = set_at(sv, iv, N, nh);
    const int64_t N1 = N, N2 = (int64_t)N * N;
    // element e of line u: base(u) + e * stride
    int64_t stride;
    if (axis == 0) stride = 1;
    else if (axis == 1) stride = N1;
    else stride = N2;
    auto base = [&](int u) -> int64_t {
        if (axis == 0) return (int64_t)v * N2 + (int64_t)u * N1;  // line (y = u, z = v)
        if (axis == 1) return (int64_t)v * N2 + u;                // line (x = u, z = v)
        return (int64_t)v * N1 + u;                               // line (x = u, y = v)
    };
    const int nl = min(PER, cu - iu0);
    const int LS = lp(N) + 1;  // line stride in LDS: the +1 spreads the PER lines of a transposed copy over the banks
    const int log2PER = __builtin_ctz(PER);  // N and PER are powers of two: shifts, not divisions
    // copy in: axis 0 with the element index fastest, axes 1 and 2 with the line index fastest
    for (int t = threadIdx.x; t < PER * N; t += blockDim.x) {
        int li, e;
        if (axis == 0) { li = t >> log2N; e = t & (N - 1); }
        else { li = t & (PER - 1); e = t >> log2PER; }
        double2 val = make_double2(0.0, 0.0);
        if (li < nl && set_has(ld, e, N, nh)) {
            val = a[base(set_at(su, iu0 + li, N, nh)) + e * stride];
            if (inv) val.y = -val.y;
        }
        sh3[(int64_t)li * LS + lp(e)] = val;
    }
    __syncthreads();
    const int li = threadIdx.x / NT, lt = threadIdx.x % NT;
    fft_line_st(sh3 + (int64_t)li * LS, N, log2N, lt, NT, tw);
    for (int t = threadIdx.x; t < PER * N; t += blockDim.x) {
        int l2, e;
        if (axis == 0) { l2 = t >> log2N; e = t & (N - 1); }
        else { l2 = t & (PER - 1); e = t >> log2PER; }
        if (l2 < nl && set_has(stv, e, N, nh)) {
            double2 val = sh3[(int64_t)l2 * LS + lp(e)];
            if (inv) val.y = -val.y;
            a[base(set_at(su, iu0 + l2, N, nh)) + e * stride] = val;
        }
    }
}

// ------------------------------------------------------------------ spread / multiply / gather

// Spread, one field.  One block of SW waves per tile of ST^3 base cells (a point's base cell
// is its first tap cell); the tile's footprint of F^3 grid points, F = ST + 2m - 1, is
// accumulated in LDS.  The footprint's z planes are split among the waves (wave w owns a
// contiguous range of planes); every wave takes the tile's points one after the other in
// sorted order, its lanes the point's (a, b) taps, each lane adding the taps c whose plane
// lies in the wave's range.  Each LDS value is thus updated by one wave only, in a fixed
// order of points (no atomics, no races), and the footprint is written to the tile's own
// slot of tileout [tile][F^3]; k3_fold adds the overlapping footprints.
constexpr int ST = 6;
constexpr int SW = 4;

__global__ void __launch_bounds__(64 * SW) k3_spread_tile(const double *__restrict__ taps,
                                                          const uint32_t *__restrict__ key,
                                                          const uint32_t *__restrict__ cstart,
                                                          const double *__restrict__ val, Map3 mp, int ntx, int nty,
                                                          double *__restrict__ tileout)
{
    extern __shared__ double acc[];
    const int M2 = 2 * mp.m, F = ST + M2 - 1, F2 = F * F, F3 = F2 * F;
    const int t = blockIdx.x, tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
    const int ex = mp.ext[0], ey = mp.ext[1];
    const int nbx = ex - M2 + 1, nby = ey - M2 + 1, nbz = mp.ext[2] - M2 + 1;
    const int x0 = tx * ST, y0 = ty * ST, z0 = tz * ST;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int pz0 = (wv * F) / SW, pz1 = ((wv + 1) * F) / SW;  // this wave's footprint planes
    for (int i = threadIdx.x; i < F3; i += 64 * SW) acc[i] = 0.0;
    // this lane's (a, b) taps: e = lane + 64 r < (2m)^2 <= 256
    int ne = 0, ea[4], eb[4];
    for (int e = lane; e < M2 * M2; e += 64) {
        ea[ne] = e % M2;
        eb[ne] = e / M2;
        ++ne;
    }
    __syncthreads();
    const int x1 = min(x0 + ST, nbx);
    constexpr int CMAX = (ST + 2 * MAXM - 1 + SW - 1) / SW;  // planes per wave: at most ceil((ST + 2m - 1)/SW)
    for (int dz = 0; dz < ST && z0 + dz < nbz; ++dz) {
        const int c0 = max(0, pz0 - dz), c1 = min(M2, pz1 - dz);  // taps c landing in the wave's planes
        if (c0 >= c1) continue;                                   // uniform over the wave
        for (int dy = 0; dy < ST && y0 + dy < nby; ++dy) {
            const int64_t row = ((int64_t)(z0 + dz) * ey + (y0 + dy)) * ex;
            const uint32_t j0 = cstart[row + x0], j1 = cstart[row + x1];
            for (uint32_t j = j0; j < j1; ++j) {
                const int lx = (int)(key[j] - (uint32_t)row) - x0;
                const double *tp = taps + (int64_t)j * 3 * M2;
                const double v = val[j];
                double tzc[CMAX];
#pragma unroll
                for (int k = 0; k < CMAX; ++k) tzc[k] = c0 + k < c1 ? tp[2 * M2 + c0 + k] : 0.0;
                for (int r = 0; r < ne; ++r) {
                    const int aa = ea[r], bb = eb[r];
                    const double wab = tp[aa] * tp[M2 + bb] * v;
                    double *ap = acc + ((dz + c0) * F + dy + bb) * F + lx + aa;
                    double cur[CMAX];
#pragma unroll
                    for (int k = 0; k < CMAX; ++k)
                        if (c0 + k < c1) cur[k] = ap[k * F2];
#pragma unroll
                    for (int k = 0; k < CMAX; ++k)
                        if (c0 + k < c1) ap[k * F2] = fma(wab, tzc[k], cur[k]);
                }
            }
        }
    }
    __syncthreads();
    double *o = tileout + (int64_t)t * F3;
    for (int i = threadIdx.x; i < F3; i += 64 * SW) o[i] = acc[i];
}

// Grid value at every data-window point: the sum of the footprints of the tiles that reach
// it, in tile order, written into the G^3 grid at the window offset: as (value, 0) for
// comp 0, into the imaginary part alone for comp 1 (a second real field packed into the
// same complex grid, after its comp-0 field).
__global__ void k3_fold(const double *__restrict__ tileout, Map3 mp, int ntx, int nty, int ntz, int G,
                        double2 *__restrict__ g, int comp)
{
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int ex = mp.ext[0], ey = mp.ext[1], ez = mp.ext[2];
    if (idx >= (int64_t)ex * ey * ez) return;
    const int kx = (int)(idx % ex), ky = (int)((idx / ex) % ey), kz = (int)(idx / ((int64_t)ex * ey));
    const int F = ST + 2 * mp.m - 1, F2 = F * F, F3 = F2 * F;
    // tiles t with t ST <= k <= t ST + F - 1: t from ceil((k - F + 1) / ST) (at least 0) to k / ST
    auto lo = [&](int k) { return k - F + 1 <= 0 ? 0 : (k - F + ST) / ST; };
    const int txl = lo(kx), tyl = lo(ky), tzl = lo(kz);
    const int txh = min(ntx - 1, kx / ST), tyh = min(nty - 1, ky / ST), tzh = min(ntz - 1, kz / ST);
    double s = 0.0;
    for (int tz = tzl; tz <= tzh; ++tz)
        for (int ty = tyl; ty <= tyh; ++ty) {
            const int64_t tb = ((int64_t)tz * nty + ty) * ntx;
            const int oz = kz - tz * ST, oy = ky - ty * ST;
            for (int tx = txl; tx <= txh; ++tx) s += tileout[(tb + tx) * F3 + (oz * F + oy) * F + (kx - tx * ST)];
        }
    const int64_t o = ((int64_t)(kz + mp.wlo[2]) * G + (ky + mp.wlo[1])) * G + (kx + mp.wlo[0]);
    if (comp == 0) g[o] = make_double2(s, 0.0);
    else reinterpret_cast<double *>(g)[2 * o + 1] = s;
}

__device__ __forceinline__ int w_idx(int nh, int a0, int a1, int a2)
{
    return (a0 * (nh + 1) + a1) * (nh + 1) + a2;
}

// forward multiply over the band^3 frequencies only (the inverse passes read nothing else):
// T1 = W F + i (-2 pi i l_z W F) (phi + i H_z), T2 = (-2 pi i l_x W F) + i (-2 pi i l_y W F)
__global__ void k3_mul_fwd(const double2 *__restrict__ F, double2 *__restrict__ T1, double2 *__restrict__ T2, int G,
                           int nh, const double *__restrict__ W)
{
    const int cb = 2 * nh + 1;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)cb * cb * cb) return;
    const int ix = (int)(idx % cb), iy = (int)((idx / cb) % cb), iz = (int)(idx / ((int64_t)cb * cb));
    const int lx = ix <= nh ? ix : ix - cb, ly = iy <= nh ? iy : iy - cb, lz = iz <= nh ? iz : iz - cb;
    const int64_t o = ((int64_t)(lz < 0 ? lz + G : lz) * G + (ly < 0 ? ly + G : ly)) * G + (lx < 0 ? lx + G : lx);
    const double wv = W[w_idx(nh, abs(lz), abs(ly), abs(lx))];
    const double2 f = make_double2(wv * F[o].x, wv * F[o].y);
    const double tp = 2.0 * PI;
    // (-2 pi i l) f = (2 pi l f.y, -2 pi l f.x)
    const double2 hx = make_double2(tp * lx * f.y, -tp * lx * f.x);
    const double2 hy = make_double2(tp * ly * f.y, -tp * ly * f.x);
    const double2 hz = make_double2(tp * lz * f.y, -tp * lz * f.x);
    T1[o] = make_double2(f.x - hz.y, f.y + hz.x);   // f + i hz
    T2[o] = make_double2(hx.x - hy.y, hx.y + hy.x); // hx + i hy
}

// adjoint multiply over the band^3 frequencies, T = sum_d (2 pi i l_d) W F_d, with the three
// fields in two transforms: Z = F0 + i F1 (two real fields packed in one complex grid) and F2.  A real field's spectrum is Hermitian, so at each band frequency
// F0(l) = (Z(l) + conj Z(-l)) / 2 and F1(l) = (Z(l) - conj Z(-l)) / 2i; T goes to its own
// grid (the thread of l reads Z at -l too).
__global__ void k3_mul_adj_packed(const double2 *__restrict__ Z, const double2 *__restrict__ F2,
                                  double2 *__restrict__ T, int G, int nh, const double *__restrict__ W)
{
    const int cb = 2 * nh + 1;
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)cb * cb * cb) return;
    const int ix = (int)(idx % cb), iy = (int)((idx / cb) % cb), iz = (int)(idx / ((int64_t)cb * cb));
    const int lx = ix <= nh ? ix : ix - cb, ly = iy <= nh ? iy : iy - cb, lz = iz <= nh ? iz : iz - cb;
    auto at = [G](int x, int y, int z) {
        return ((int64_t)(z < 0 ? z + G : z) * G + (y < 0 ? y + G : y)) * G + (x < 0 ? x + G : x);
    };
    const int64_t o = at(lx, ly, lz), om = at(-lx, -ly, -lz);
    const double wv = W[w_idx(nh, abs(lz), abs(ly), abs(lx))] * 2.0 * PI;
    const double2 z = Z[o], zm = Z[om], c = F2[o];
    const double2 a = make_double2(0.5 * (z.x + zm.x), 0.5 * (z.y - zm.y));   // F0(l)
    const double2 b = make_double2(0.5 * (z.y + zm.y), -0.5 * (z.x - zm.x));  // F1(l)
    // (i l) f = (-l f.y, l f.x)
    const double sx = -(lx * a.y + ly * b.y + lz * c.y), sy = lx * a.x + ly * b.x + lz * c.x;
    T[o] = make_double2(wv * sx, wv * sy);
}

// Far values at the points of a set, LG lanes per point (8 when 2m <= 8, else 16): lane a
// takes the x tap a (a < 2m), every lane loops over the (b, c) taps, reading 2m consecutive
// grid values per row across the point's lanes; the LG partial sums are then added by a
// butterfly within the group (a fixed order).  nout = 1: out[k] = re A; nout = 4 (forward): A = phi + i H_z,
// B = H_x + i H_y -> out[f][k] for f = phi, H_x, H_y, H_z.
template <int LG>
__global__ void __launch_bounds__(256) k3_gather(const double *__restrict__ taps, const uint32_t *__restrict__ key,
                                                 int64_t N, Map3 mp, const double2 *__restrict__ A,
                                                 const double2 *__restrict__ B, int nout, int G, double *__restrict__ out)
{
    const int64_t k = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / LG;
    const int a = threadIdx.x % LG;
    if (k >= N) return;  // the whole group of LG leaves together
    const int M2 = 2 * mp.m;
    const bool act = a < M2;
    const uint32_t kk = key[k];
    const int b0 = (int)(kk % (uint32_t)mp.ext[0]), b1 = (int)((kk / (uint32_t)mp.ext[0]) % (uint32_t)mp.ext[1]);
    const int b2 = (int)(kk / ((uint32_t)mp.ext[0] * (uint32_t)mp.ext[1]));
    const double *tp = taps + k * 3 * M2;
    const double txa = act ? tp[a] : 0.0;
    double ty[LG], tz[LG];  // the point's y and z taps in registers (2m <= LG)
#pragma unroll
    for (int i = 0; i < LG; ++i) {
        ty[i] = i < M2 ? tp[M2 + i] : 0.0;
        tz[i] = i < M2 ? tp[2 * M2 + i] : 0.0;
    }
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    if (act) {
        const int64_t xo = (int64_t)b0 + mp.wlo[0] + a;
#pragma unroll
        for (int c = 0; c < LG; ++c) {
            if (c >= M2) break;
            const double wz = txa * tz[c];
            const int64_t zrow = ((int64_t)(b2 + c + mp.wlo[2]) * G + (b1 + mp.wlo[1])) * G + xo;
#pragma unroll
            for (int b = 0; b < LG; b += 2) {  // 2m is even: two rows per trip, loads first
                if (b >= M2) break;
                const double w0 = wz * ty[b], w1 = wz * ty[b + 1];
                const int64_t o = zrow + (int64_t)b * G;
                const double2 u0 = A[o], u1 = A[o + G];
                if (nout == 4) {
                    const double2 v0 = B[o], v1 = B[o + G];
                    acc1 = fma(w0, u0.y, acc1);
                    acc2 = fma(w0, v0.x, acc2);
                    acc3 = fma(w0, v0.y, acc3);
                    acc1 = fma(w1, u1.y, acc1);
                    acc2 = fma(w1, v1.x, acc2);
                    acc3 = fma(w1, v1.y, acc3);
                }
                acc0 = fma(w0, u0.x, acc0);
                acc0 = fma(w1, u1.x, acc0);
            }
        }
    }
    for (int s = LG / 2; s > 0; s >>= 1) {
        acc0 += __shfl_xor(acc0, s, LG);
        if (nout == 4) {
            acc1 += __shfl_xor(acc1, s, LG);
            acc2 += __shfl_xor(acc2, s, LG);
            acc3 += __shfl_xor(acc3, s, LG);
        }
    }
    if (a != 0) return;
    if (nout == 4) {
        out[k] = acc0;
        out[N + k] = acc2;
        out[2 * N + k] = acc3;
        out[3 * N + k] = acc1;
    } else {
        out[k] = acc0;
    }
}

// The same far values by tiles, for the grids whose tile footprints fit GATHER_TILE_LDS:
// one block per tile of ST^3 base cells (the spread's tiles) stages the tile's footprint
// of the grid(s), F^3 values with F = ST + 2m - 1, in LDS once, then LG lanes per point of
// the tile (lane a takes the x tap a) read the (b, c) rows from LDS in k3_gather's order
// and add their partial sums by the same butterfly, so the results are the same bits.
// The points of the tile are the ST^2 base-cell row runs of the sorted set, taken through
// their prefix sums.
constexpr int GATHER_TILE_LDS = 80 << 10;
inline size_t gather_tile_lds(int m, int ngrid)
{
    const size_t F = ST + 2 * m - 1;
    return F * F * F * sizeof(double2) * ngrid;
}

template <int LG, int NOUT>
__global__ void __launch_bounds__(256) k3_gather_tile(const double *__restrict__ taps, const uint32_t *__restrict__ key,
                                                      const uint32_t *__restrict__ cstart, int64_t N, Map3 mp, int ntx,
                                                      int nty, const double2 *__restrict__ A,
                                                      const double2 *__restrict__ B, int G, double *__restrict__ out)
{
    extern __shared__ double2 gsh[];  // [NOUT == 4 ? 2 : 1][F^3]
    __shared__ uint32_t rs[ST * ST], rp[ST * ST + 1];
    const int M2 = 2 * mp.m, F = ST + M2 - 1, F2 = F * F, F3 = F2 * F;
    const int t = blockIdx.x, tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
    const int ex = mp.ext[0], ey = mp.ext[1], ez = mp.ext[2];
    const int nbx = ex - M2 + 1, nby = ey - M2 + 1, nbz = ez - M2 + 1;
    const int x0 = tx * ST, y0 = ty * ST, z0 = tz * ST;
    if (threadIdx.x < ST * ST) {  // the tile's base-cell rows (dz, dy): their runs of points
        const int dz = threadIdx.x / ST, dy = threadIdx.x % ST;
        uint32_t s0 = 0, cnt = 0;
        if (z0 + dz < nbz && y0 + dy < nby) {
            const int64_t row = ((int64_t)(z0 + dz) * ey + (y0 + dy)) * ex;
            s0 = cstart[row + x0];
            cnt = cstart[row + min(x0 + ST, nbx)] - s0;
        }
        rs[threadIdx.x] = s0;
        rp[threadIdx.x + 1] = cnt;
    }
    // footprint: grid points (x0 + fx, y0 + fy, z0 + fz) of the window (none beyond it)
    for (int i = threadIdx.x; i < F3; i += blockDim.x) {
        const int fz = i / F2, fy = (i / F) % F, fx = i % F;
        double2 va = make_double2(0.0, 0.0), vb = va;
        if (x0 + fx < ex && y0 + fy < ey && z0 + fz < ez) {
            const int64_t o = ((int64_t)(z0 + fz + mp.wlo[2]) * G + (y0 + fy + mp.wlo[1])) * G + (x0 + fx + mp.wlo[0]);
            va = A[o];
            if (NOUT == 4) vb = B[o];
        }
        gsh[i] = va;
        if (NOUT == 4) gsh[F3 + i] = vb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        rp[0] = 0;
        for (int r = 1; r <= ST * ST; ++r) rp[r] += rp[r - 1];
    }
    __syncthreads();
    const uint32_t total = rp[ST * ST];
    const int a = threadIdx.x % LG, ngrp = blockDim.x / LG;
    const bool act = a < M2;
    // a group's lanes share idx, so every shuffle below runs with its whole group active
    for (uint32_t idx = threadIdx.x / LG; idx < total; idx += ngrp) {
        int lo = 0, hi = ST * ST - 1;  // the row of idx: the largest r with rp[r] <= idx (a non-empty row)
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rp[mid] <= idx) lo = mid;
            else hi = mid - 1;
        }
        const int64_t k = (int64_t)rs[lo] + (idx - rp[lo]);
        const uint32_t kk = key[k];
        const int lx = (int)(kk % (uint32_t)ex) - x0, ly = (int)((kk / (uint32_t)ex) % (uint32_t)ey) - y0;
        const int lz = (int)(kk / ((uint32_t)ex * (uint32_t)ey)) - z0;
        const double *tp = taps + k * 3 * M2;
        const double txa = act ? tp[a] : 0.0;
        double ty[LG], tz[LG];  // the point's y and z taps in registers (2m <= LG)
#pragma unroll
        for (int i = 0; i < LG; ++i) {
            ty[i] = i < M2 ? tp[M2 + i] : 0.0;
            tz[i] = i < M2 ? tp[2 * M2 + i] : 0.0;
        }
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
        if (act) {
#pragma unroll
            for (int c = 0; c < LG; ++c) {
                if (c >= M2) break;
                const double wz = txa * tz[c];
                const int zrow = ((lz + c) * F + ly) * F + lx + a;
#pragma unroll
                for (int b = 0; b < LG; b += 2) {
                    if (b >= M2) break;
                    const double w0 = wz * ty[b], w1 = wz * ty[b + 1];
                    const int o = zrow + b * F;
                    const double2 u0 = gsh[o], u1 = gsh[o + F];
                    if (NOUT == 4) {
                        const double2 v0 = gsh[F3 + o], v1 = gsh[F3 + o + F];
                        acc1 = fma(w0, u0.y, acc1);
                        acc2 = fma(w0, v0.x, acc2);
                        acc3 = fma(w0, v0.y, acc3);
                        acc1 = fma(w1, u1.y, acc1);
                        acc2 = fma(w1, v1.x, acc2);
                        acc3 = fma(w1, v1.y, acc3);
                    }
                    acc0 = fma(w0, u0.x, acc0);
                    acc0 = fma(w1, u1.x, acc0);
                }
            }
        }
        for (int sft = LG / 2; sft > 0; sft >>= 1) {
            acc0 += __shfl_xor(acc0, sft, LG);
            if (NOUT == 4) {
                acc1 += __shfl_xor(acc1, sft, LG);
                acc2 += __shfl_xor(acc2, sft, LG);
                acc3 += __shfl_xor(acc3, sft, LG);
            }
        }
        if (a == 0) {
            if (NOUT == 4) {
                out[k] = acc0;
                out[N + k] = acc2;
                out[2 * N + k] = acc3;
                out[3 * N + k] = acc1;
            } else {
                out[k] = acc0;
            }
        }
    }
}

// ------------------------------------------------------------------ near field + final

struct Near3 {
    double e2g, inv_e2g;   // (eps_I G)^2 and its inverse: x = r^2 / (eps_I G)^2 with r in grid units
    double a[MAXP], da[MAXP];  // T_I(x) = sum a_k x^k; D(x) = sum da_k x^k, da_k = (k+1) a_{k+1}
    double cphi;           // G/(4 pi): K(r/G) = cphi / r for r in grid units
    double cD;             // 2/((eps_I G)^2 G)
    double G2;             // G^2: the H sums are in grid units
    int p, R;
    double s;
    int hb[3], nh[3];      // home block edge (cells) and home block counts per axis
};

// Near field.  One block of NB threads per home block of hb[0] x hb[1] x hb[2] base cells
// of the output ("home") set.  The cells of the input set that can hold a point within
// eps_I of the home block form, per (z, y) row, one run of cells, hence one contiguous run
// of sorted points; the runs are concatenated (block prefix sum) and the block's threads
// take the candidates of the concatenation one each (coalesced loads), each against the
// home points of the block, KC at a time (positions in registers; 4 in the forward kernel,
// whose four sums per home point would otherwise hold it to 3 waves per SIMD, 8 in the
// adjoint, which has one sum and gains more from reusing each candidate), with per-home-point
// partial sums in registers.  The partial sums are added over the block in a fixed order
// (wave butterflies, then the waves in order), so the result does not depend on timing.
// Positions are in grid units relative to the data window: base cell + in-cell fraction.
// Per pair (r = |d| in grid units, x = r^2/(eps_I G)^2, zone r < eps_I G):
//   phi += s_j (cphi/r - T_I(x)),    H-sum += s_j (1/(4 pi r^3) + cD D(x)) d
// (H = s^2 (far + G^2 H-sum)); a pair at distance 0 adds -s_j a_0 to phi instead.  The
// adjoint (home = sources, input = targets with payload V) adds -(1/(4 pi r^3) + cD D(x)) V.d.
// 1/r: hardware reciprocal square root estimate and two Newton steps.
constexpr int NB = 256;
constexpr int KC_FWD = 4, KC_ADJ = 8;
constexpr int RMAP = 8192;  // candidates per block whose row is tabulated in LDS (more: binary search)

__device__ __forceinline__ double rsqrt64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// exclusive prefix over the block (NB threads); returns the prefix of v, *total the sum
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t *sh, uint32_t *total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < NB; off <<= 1) {
        const uint32_t o = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += o;
        __syncthreads();
    }
    const uint32_t incl = sh[t];
    *total = sh[NB - 1];
    __syncthreads();
    return incl - v;
}

template <bool ADJ, int P>
__global__ void __launch_bounds__(NB) k3_near(const double4 *__restrict__ pos_out, const uint32_t *__restrict__ cs_out,
                                              const uint32_t *__restrict__ perm_out, int64_t n_out,
                                              const double4 *__restrict__ pos_in, const uint32_t *__restrict__ cs_in,
                                              const double *__restrict__ pay, int64_t n_in, Map3 mp, Near3 nr,
                                              const double *__restrict__ far, const double *__restrict__ w_out,
                                              double *__restrict__ o_phi, double *__restrict__ o_H)
{
    extern __shared__ uint32_t nsh[];
    constexpr int NV = ADJ ? 1 : 4;
    constexpr int KC = ADJ ? KC_ADJ : KC_FWD;
    const int ex = mp.ext[0], ey = mp.ext[1];
    const int M2 = 2 * mp.m;
    const int nbx = ex - M2 + 1, nby = ey - M2 + 1, nbz = mp.ext[2] - M2 + 1;
    const int b = blockIdx.x;
    const int hx0 = (b % nr.nh[0]) * nr.hb[0], hy0 = ((b / nr.nh[0]) % nr.nh[1]) * nr.hb[1];
    const int hz0 = (b / (nr.nh[0] * nr.nh[1])) * nr.hb[2];
    const int hx1 = min(hx0 + nr.hb[0], nbx);
    const int R = nr.R;
    const int zlo = max(hz0 - R, 0), zhi = min(hz0 + nr.hb[2] - 1 + R, nbz - 1);
    const int ylo = max(hy0 - R, 0), yhi = min(hy0 + nr.hb[1] - 1 + R, nby - 1);
    const int nyr = yhi - ylo + 1, nrows = (zhi - zlo + 1) * nyr;
    // LDS: scan scratch [NB], home segments, row starts and prefixes [nrows + 1], home chunk, reduction
    uint32_t *scan = nsh;
    uint32_t *hseg = scan + NB;                   // [8] starts, [9] prefixes
    uint32_t *hpre = hseg + 8;
    uint32_t *rstart = hpre + 9;
    uint32_t *rpre = rstart + nrows;
    double *red = reinterpret_cast<double *>(nsh + ((NB + 17 + 2 * nrows + 1 + 1) & ~1));  // [NB/64][KC][NV]
    uint16_t *rmap = reinterpret_cast<uint16_t *>(red + (NB / 64) * (KC_FWD * 4 > KC_ADJ ? KC_FWD * 4 : KC_ADJ));  // [RMAP]
    const int t = threadIdx.x;

    // home points: one run per home row (at most 8 rows: hb[1] hb[2] <= 8)
    const int nseg = nr.hb[1] * nr.hb[2];
    if (t < nseg) {
        const int y = hy0 + t % nr.hb[1], z = hz0 + t / nr.hb[1];
        uint32_t s0 = 0, cnt = 0;
        if (y < nby && z < nbz) {
            const int64_t rb = ((int64_t)z * ey + y) * ex;
            s0 = cs_out[rb + hx0];
            cnt = cs_out[rb + hx1] - s0;
        }
        hseg[t] = s0;
        hpre[t + 1] = cnt;
    }
    __syncthreads();
    if (t == 0) {
        hpre[0] = 0;
        for (int s = 1; s <= nseg; ++s) hpre[s] += hpre[s - 1];
    }
    __syncthreads();
    const uint32_t nhome = hpre[nseg];
    if (nhome == 0) return;  // uniform

    // candidate runs per input row (z, y): cells whose x extent meets [hx0 - w, hx1 + w]
    const double e2 = nr.e2g;
    const int per = (nrows + NB - 1) / NB;
    uint32_t mysum = 0;
    for (int r = t * per; r < min(nrows, (t + 1) * per); ++r) {
        const int z = zlo + r / nyr, y = ylo + r % nyr;
        const double gz = z >= hz0 + nr.hb[2] ? (double)(z - hz0 - nr.hb[2]) : (z + 1 <= hz0 ? (double)(hz0 - z - 1) : 0.0);
        const double gy = y >= hy0 + nr.hb[1] ? (double)(y - hy0 - nr.hb[1]) : (y + 1 <= hy0 ? (double)(hy0 - y - 1) : 0.0);
        const double h2 = e2 - gz * gz - gy * gy;
        uint32_t s0 = 0, cnt = 0;
        if (h2 > 0.0) {
            const double w = sqrt(h2);
            const int xa = max((int)floor((double)hx0 - w), 0);
            const int xb = min((int)floor((double)hx1 + w), nbx - 1);
            if (xa <= xb) {
                const int64_t rb = ((int64_t)z * ey + y) * ex;
                s0 = cs_in[rb + xa];
                cnt = cs_in[rb + xb + 1] - s0;
            }
        }
        rstart[r] = s0;
        rpre[r] = cnt;
        mysum += cnt;
    }
    uint32_t total;
    uint32_t run = block_scan(mysum, scan, &total);
    for (int r = t * per; r < min(nrows, (t + 1) * per); ++r) {
        const uint32_t cnt = rpre[r];
        rpre[r] = run;
        run += cnt;
    }
    if (t == 0) rpre[nrows] = total;
    __syncthreads();
    // the row of every candidate, so that a thread finds its candidate's row with one read
    // (block-uniform choice; a block with more candidates searches the row prefixes)
    const bool use_map = total <= (uint32_t)RMAP;
    if (use_map) {
        for (int r = t * per; r < min(nrows, (t + 1) * per); ++r)
            for (uint32_t i = rpre[r]; i < rpre[r + 1]; ++i) rmap[i] = (uint16_t)r;
        __syncthreads();
    }

    const double a0 = nr.a[0];
    for (uint32_t kc0 = 0; kc0 < nhome; kc0 += KC) {
        const int kn = (int)min((uint32_t)KC, nhome - kc0);  // home points in this chunk (block-uniform)
        // this chunk's home positions (a far sentinel for empty slots never enters the zone)
        double hx[KC], hy[KC], hz[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            const uint32_t kk = kc0 + k;
            hx[k] = hy[k] = hz[k] = 1e30;
            if (kk < nhome) {
                int s = 0;
                while (s + 1 < nseg && hpre[s + 1] <= kk) ++s;
                const double4 h = pos_out[hseg[s] + (kk - hpre[s])];
                hx[k] = h.x;
                hy[k] = h.y;
                hz[k] = h.z;
            }
        }
        double acc[KC][NV];
#pragma unroll
        for (int k = 0; k < KC; ++k)
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[k][v] = 0.0;
        for (uint32_t idx = t; idx < total; idx += NB) {
            int lo = 0, hi = nrows - 1;  // largest row with rpre <= idx (a non-empty row)
            if (use_map) {
                lo = rmap[idx];
            } else {
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (rpre[mid] <= idx) lo = mid; else hi = mid - 1;
                }
            }
            const uint32_t j = rstart[lo] + (idx - rpre[lo]);
            const double4 q = pos_in[j];
            double w0, w1 = 0.0, w2 = 0.0;
            if (ADJ) {
                w0 = pay[j];
                w1 = pay[n_in + j];
                w2 = pay[2 * n_in + j];
            } else {
                w0 = pay[j];
            }
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                if (k >= kn) break;  // uniform: a short last chunk costs only its own pairs
                const double dx = hx[k] - q.x, dy = hy[k] - q.y, dz = hz[k] - q.z;
                const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                const bool inz = r2 < e2;
                const bool pos = r2 > 0.0;
                // x is capped at the zone edge so that pairs outside (and the sentinel) stay finite;
                // their terms are masked below
                const double x = fmin(r2 * nr.inv_e2g, 1.0);
                const double ri = rsqrt64(fmax(r2, 1e-200));
                double d = 0.0;
                if (P >= 2) {
                    d = nr.da[P - 2];
#pragma unroll
                    for (int i = P - 3; i >= 0; --i) d = fma(d, x, nr.da[i]);
                }
                const double g = fma(INV_4PI * ri, ri * ri, nr.cD * d);
                if (!ADJ) {
                    double tt = nr.a[P - 1];
#pragma unroll
                    for (int i = P - 2; i >= 0; --i) tt = fma(tt, x, nr.a[i]);
                    const double ph = pos ? fma(nr.cphi, ri, -tt) : -a0;
                    const double sp = inz ? w0 : 0.0;
                    const double sh = (inz && pos) ? w0 * g : 0.0;
                    acc[k][0] = fma(sp, ph, acc[k][0]);
                    acc[k][1] = fma(sh, dx, acc[k][1]);
                    acc[k][2] = fma(sh, dy, acc[k][2]);
                    acc[k][3] = fma(sh, dz, acc[k][3]);
                } else {
                    const double gm = (inz && pos) ? g : 0.0;
                    acc[k][0] = fma(-gm, fma(w0, dx, fma(w1, dy, w2 * dz)), acc[k][0]);
                }
            }
        }
        // block sums in a fixed order: butterflies within each wave, then the waves in order
        const int lane = t & 63, wv = t >> 6;
#pragma unroll
        for (int k = 0; k < KC; ++k)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double s = acc[k][v];
                for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
                if (lane == 0) red[(wv * KC + k) * NV + v] = s;
            }
        __syncthreads();
        if (t < KC) {
            const uint32_t kk = kc0 + t;
            if (kk < nhome) {
                double sv[NV];
                for (int v = 0; v < NV; ++v) {
                    double s = 0.0;
                    for (int w = 0; w < NB / 64; ++w) s += red[(w * KC + t) * NV + v];
                    sv[v] = s;
                }
                int s = 0;
                while (s + 1 < nseg && hpre[s + 1] <= kk) ++s;
                const uint32_t i = hseg[s] + (kk - hpre[s]);
                const uint32_t o = perm_out[i];
                const double s1 = nr.s, s2 = s1 * s1, G2 = nr.G2;
                if (!ADJ) {
                    if (o_phi) o_phi[o] = s1 * (far[i] + sv[0]);
                    if (o_H) {
                        o_H[3 * (int64_t)o] = s2 * fma(G2, sv[1], far[n_out + i]);
                        o_H[3 * (int64_t)o + 1] = s2 * fma(G2, sv[2], far[2 * n_out + i]);
                        o_H[3 * (int64_t)o + 2] = s2 * fma(G2, sv[3], far[3 * n_out + i]);
                    }
                } else {
                    o_phi[o] = w_out[i] * s2 * fma(G2, sv[0], far[i]);
                }
            }
        }
        __syncthreads();
    }
}

inline size_t near3_lds_bytes(int nrows)
{
    const size_t words = ((size_t)NB + 17 + 2 * (size_t)nrows + 1 + 1) & ~(size_t)1;
    return words * 4 + (size_t)(NB / 64) * std::max(KC_FWD * 4, KC_ADJ) * sizeof(double) + (size_t)RMAP * 2;
}

// values in sorted order: out[f][k] = (w_k) in[perm_k][f] (w NULL: 1), nf components per point
__global__ void k3_values(const double *__restrict__ in, const double *__restrict__ w, const uint32_t *__restrict__ perm,
                          int64_t n, int nf, double *__restrict__ out)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t i = perm[k];
    for (int f = 0; f < nf; ++f) out[f * n + k] = (w ? w[k] : 1.0) * in[(int64_t)i * nf + f];
}

// Debug validation of one binned set (FEMNFFT_DEBUG_CHECKS): keys sorted and inside the cell
// table, cell starts consistent with the keys, each packed position inside its key's cell
// (closed: base cell + fraction may round up to the next integer),
// perm a permutation of [0, n) (cnt: n counters, zeroed by the caller's k3_zero32)
__global__ void k3_zero32(uint32_t *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k3_check_bins(const uint32_t *__restrict__ key, const uint32_t *__restrict__ perm,
                              const uint32_t *__restrict__ cstart, const double4 *__restrict__ pos, int64_t n,
                              int ex, int ey, int64_t ncell, uint32_t *__restrict__ cnt, uint32_t *__restrict__ bad)
{
    uint32_t v = 0;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t kk = key[k];
        if ((int64_t)kk >= ncell) {
            ++v;
        } else {
            if ((int64_t)cstart[kk] > k || (int64_t)cstart[kk + 1] <= k) ++v;
            const double4 q = pos[k];
            const int b0 = (int)(kk % (uint32_t)ex), b1 = (int)((kk / (uint32_t)ex) % (uint32_t)ey);
            const int b2 = (int)(kk / ((uint32_t)ex * (uint32_t)ey));
            // base cell + fraction may round up to the next integer: the cell's closed extent
            if (!(q.x >= b0 && q.x <= b0 + 1 && q.y >= b1 && q.y <= b1 + 1 && q.z >= b2 && q.z <= b2 + 1)) ++v;
        }
        if (k + 1 < n && key[k + 1] < kk) ++v;
        const uint32_t i = perm[k];
        if ((int64_t)i >= n) ++v;
        else atomicAdd(&cnt[i], 1u);
    }
    if (v) atomicAdd(bad, v);
}

__global__ void k3_check_perm(const uint32_t *__restrict__ cnt, int64_t n, uint32_t *__restrict__ bad)
{
    uint32_t v = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v += cnt[i] != 1u ? 1u : 0u;
    if (v) atomicAdd(bad, v);
}

__global__ void k3_fill(double *p, int64_t n, double v)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

inline int nbk(int64_t n) { return (int)std::max<int64_t>(1, (n + NT - 1) / NT); }

}  // namespace fn3

using namespace fn3;

#define F3_ERR(c, code, msg) \
    do {                     \
        (c)->err = (msg);    \
        return (code);       \
    } while (0)
#define F3_HIP(c, call)                                                                       \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            (c)->err = std::string("HIP error in ") + #call + ": " + hipGetErrorString(e_);   \
            return FN_E_DEVICE;                                                               \
        }                                                                                     \
    } while (0)
#define F3_LAUNCH(c) F3_HIP(c, hipGetLastError())

namespace {

constexpr size_t PROF3_MAX = 4096;

int prof3_begin(fn3_ctx *c, int st)
{
    if (!c->prof_on || stream_capturing(c->stream)) return -1;
    if (c->prof_next >= PROF3_MAX) {
        c->prof.dropped += 1;
        return -1;
    }
    const size_t i = c->prof_next++;
    c->prof_stage[i] = st;
    hipEventRecord(c->prof_ev[2 * i], c->stream);
    return (int)i;
}

void prof3_end(fn3_ctx *c, int i)
{
    if (i >= 0) hipEventRecord(c->prof_ev[2 * i + 1], c->stream);
}

struct Layout3 {
    size_t total = 0, off_W = 0, off_twG = 0, off_ctab = 0, off_key[2] = {0, 0}, off_perm[2] = {0, 0},
           off_cs[2] = {0, 0}, off_fr[2] = {0, 0}, off_taps[2] = {0, 0}, off_w = 0, off_val = 0, off_aval = 0,
           off_grid[3] = {0, 0, 0},
           off_far = 0, off_red = 0, off_skey = 0, off_sval = 0, off_hist = 0, off_tiles = 0;
    int64_t emax = 0;
};

Layout3 layout3(const Plan3 &P, int64_t nt, int64_t ns)
{
    Layout3 L;
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t r = o;
        o = (o + b + 255) & ~(size_t)255;
        return r;
    };
    const int nh1 = P.n / 2 + 1;
    // data window extent per axis: at most floor((1/2 - eps_B) G) + 2m + 3 cells
    L.emax = (int64_t)std::floor((0.5 - P.eps_B) * P.G) + 2 * P.m + 4;
    const int64_t ncell = L.emax * L.emax * L.emax;
    const int64_t N[2] = {std::max<int64_t>(nt, 1), std::max<int64_t>(ns, 1)};
    const int64_t nmax = std::max(N[0], N[1]);
    const int64_t G3 = (int64_t)P.G * P.G * P.G;
    L.off_W = take((size_t)nh1 * nh1 * nh1 * 8);
    L.off_twG = take((size_t)P.G * 16);
    L.off_ctab = take((size_t)P.n * 8);
    for (int s = 0; s < 2; ++s) {
        L.off_key[s] = take(N[s] * 4);
        L.off_perm[s] = take(N[s] * 4);
        L.off_cs[s] = take((size_t)(ncell + 1) * 4);
        L.off_fr[s] = take(N[s] * 32);
        L.off_taps[s] = take(N[s] * 3 * 2 * P.m * 8);
    }
    L.off_w = take(N[1] * 8);
    L.off_val = take(N[1] * 8);
    L.off_aval = take(3 * N[0] * 8);
    // three G^3 complex grids; two of them also hold the plan's (n/2 + 1)^3 cosine sums
    for (int g = 0; g < 3; ++g) L.off_grid[g] = take((size_t)G3 * 16);
    L.off_far = take(4 * nmax * 8);
    L.off_red = take(8192 * 8);
    L.off_skey = take(nmax * 4);
    L.off_sval = take(nmax * 4);
    L.off_hist = take((size_t)256 * ((nmax + 4095) / 4096) * 4);
    {  // spread tile footprints, one field
        const int64_t nt1 = (L.emax - 2 * P.m + 1 + ST - 1) / ST, F = ST + 2 * P.m - 1;
        L.off_tiles = take((size_t)(nt1 * nt1 * nt1) * (size_t)(F * F * F) * 8);
    }
    L.total = o;
    return L;
}

void bind3(fn3_ctx *c, const Layout3 &L)
{
    char *b = static_cast<char *>(c->ws);
    Buf3 &B = c->buf;
    B.W = reinterpret_cast<double *>(b + L.off_W);
    B.twG = reinterpret_cast<double2 *>(b + L.off_twG);
    B.ctab = reinterpret_cast<double *>(b + L.off_ctab);
    for (int s = 0; s < 2; ++s) {
        B.key[s] = reinterpret_cast<uint32_t *>(b + L.off_key[s]);
        B.perm[s] = reinterpret_cast<uint32_t *>(b + L.off_perm[s]);
        B.cstart[s] = reinterpret_cast<uint32_t *>(b + L.off_cs[s]);
        B.pos[s] = reinterpret_cast<double4 *>(b + L.off_fr[s]);
        B.taps[s] = reinterpret_cast<double *>(b + L.off_taps[s]);
    }
    B.w = reinterpret_cast<double *>(b + L.off_w);
    B.val = reinterpret_cast<double *>(b + L.off_val);
    B.aval = reinterpret_cast<double *>(b + L.off_aval);
    for (int g = 0; g < 3; ++g) B.grid[g] = reinterpret_cast<double2 *>(b + L.off_grid[g]);
    B.far = reinterpret_cast<double *>(b + L.off_far);
    B.red = reinterpret_cast<double *>(b + L.off_red);
    B.skey = reinterpret_cast<uint32_t *>(b + L.off_skey);
    B.sval = reinterpret_cast<uint32_t *>(b + L.off_sval);
    B.hist = reinterpret_cast<uint32_t *>(b + L.off_hist);
    B.tiles = reinterpret_cast<double *>(b + L.off_tiles);
}

constexpr int PASS_THREADS = 512;
constexpr size_t PASS_LDS = (size_t)80 << 10;

Set3 s_int(int lo, int len) { return Set3{0, lo, len}; }
Set3 s_band() { return Set3{1, 0, 0}; }

int pass3(fn3_ctx *c, double2 *a, int N, int log2N, int axis, int inv, int nh, Set3 su, Set3 sv, Set3 ld, Set3 stv,
          const double2 *tw)
{
    auto count = [&](const Set3 &s) { return s.kind == 0 ? s.len : (s.kind == 1 ? 2 * nh + 1 : N); };
    const int NT = N / FFT_EPT, PER = PASS_THREADS / NT;
    const size_t lds = (size_t)PER * (fn::fftd::lp(N) + 1) * sizeof(double2);
    if (lds > PASS_LDS) F3_ERR(c, FN_E_DEVICE, "internal: line pass LDS");
    const int cu = count(su), cv = count(sv);
    if (cu <= 0 || cv <= 0) return FN_OK;
    dim3 grid((cu + PER - 1) / PER, cv);
    k3_pass<<<grid, PASS_THREADS, lds, c->stream>>>(a, N, log2N, axis, inv, nh, su, sv, ld, stv, tw);
    F3_LAUNCH(c);
    return FN_OK;
}

// Forward transform of a grid that is zero outside the data window, keeping the band^3
// frequencies only: x lines of the window's (y, z) rows, then y lines of the band's x
// columns in the window's z planes, then z lines of band x band.
int fft3_fwd(fn3_ctx *c, double2 *a)
{
    const Plan3 &P = c->plan;
    const Geom3 &g = c->geom;
    const int nh = P.n / 2;
    const Set3 wx = s_int(g.wlo[0], g.ext[0]), wy = s_int(g.wlo[1], g.ext[1]), wz = s_int(g.wlo[2], g.ext[2]);
    int rc = pass3(c, a, P.G, P.log2G, 0, 0, nh, wy, wz, wx, s_band(), c->buf.twG);
    if (!rc) rc = pass3(c, a, P.G, P.log2G, 1, 0, nh, s_band(), wz, wy, s_band(), c->buf.twG);
    if (!rc) rc = pass3(c, a, P.G, P.log2G, 2, 0, nh, s_band(), s_band(), wz, s_band(), c->buf.twG);
    return rc;
}

// Inverse transform of a spectrum that is zero outside band^3, computing the data window only.
int fft3_inv(fn3_ctx *c, double2 *a)
{
    const Plan3 &P = c->plan;
    const Geom3 &g = c->geom;
    const int nh = P.n / 2;
    const Set3 wx = s_int(g.wlo[0], g.ext[0]), wy = s_int(g.wlo[1], g.ext[1]), wz = s_int(g.wlo[2], g.ext[2]);
    int rc = pass3(c, a, P.G, P.log2G, 2, 1, nh, s_band(), s_band(), s_band(), wz, c->buf.twG);
    if (!rc) rc = pass3(c, a, P.G, P.log2G, 1, 1, nh, s_band(), wz, s_band(), wy, c->buf.twG);
    if (!rc) rc = pass3(c, a, P.G, P.log2G, 0, 1, nh, wy, wz, s_band(), wx, c->buf.twG);
    return rc;
}

int build_plan3(fn3_ctx *c)
{
    const Plan3 &P = c->plan;
    Buf3 &B = c->buf;
    hipStream_t st = c->stream;
    F3_HIP(c, hipFuncSetAttribute((const void *)k3_pass, hipFuncAttributeMaxDynamicSharedMemorySize, (int)PASS_LDS));
    {
        const int F = ST + 2 * MAXM - 1;
        F3_HIP(c, hipFuncSetAttribute((const void *)k3_spread_tile, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      F * F * F * (int)sizeof(double)));
        const void *gk[4] = {(const void *)k3_gather_tile<8, 1>, (const void *)k3_gather_tile<8, 4>,
                             (const void *)k3_gather_tile<16, 1>, (const void *)k3_gather_tile<16, 4>};
        for (const void *k : gk)
            F3_HIP(c, hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, GATHER_TILE_LDS));
    }
    F3_HIP(c, hipMemcpyAsync(B.twG, P.twG.data(), P.twG.size() * 8, hipMemcpyHostToDevice, st));
    F3_HIP(c, hipMemcpyAsync(B.ctab, P.ctab.data(), P.ctab.size() * 8, hipMemcpyHostToDevice, st));
    double *coef = B.red, *cB = B.red + 32, *psi = B.red + 128;
    F3_HIP(c, hipMemcpyAsync(coef, P.a, sizeof(double) * MAXP, hipMemcpyHostToDevice, st));
    F3_HIP(c, hipMemcpyAsync(cB, P.cB.data(), sizeof(double) * P.cB.size(), hipMemcpyHostToDevice, st));
    F3_HIP(c, hipMemcpyAsync(psi, P.psihat.data(), sizeof(double) * P.psihat.size(), hipMemcpyHostToDevice, st));
    const int64_t nh1 = P.n / 2 + 1, nh3 = nh1 * nh1 * nh1;
    double *ha = reinterpret_cast<double *>(B.grid[0]), *hb = reinterpret_cast<double *>(B.grid[1]);
    k3_kr_samples<<<nbk(nh3), NT, 0, st>>>(ha, P.n, coef, P.p, P.eps_I, P.eps_B, cB, (int)P.cB.size());
    F3_LAUNCH(c);
    for (int axis = 0; axis < 3; ++axis) {
        k3_cos_pass<<<nbk(nh3), NT, 0, st>>>(ha, hb, P.n, axis, B.ctab);
        F3_LAUNCH(c);
        std::swap(ha, hb);
    }
    k3_make_W<<<nbk(nh3), NT, 0, st>>>(ha, P.n, psi, B.W);
    F3_LAUNCH(c);
    F3_HIP(c, hipStreamSynchronize(st));
    c->plan_ready = true;
    return FN_OK;
}

Map3 map_of(const fn3_ctx *c)
{
    Map3 mp;
    for (int d = 0; d < 3; ++d) {
        mp.c[d] = c->geom.c[d];
        mp.wlo[d] = c->geom.wlo[d];
        mp.ext[d] = c->geom.ext[d];
    }
    mp.s = c->geom.s;
    mp.G = c->plan.G;
    mp.m = c->plan.m;
    return mp;
}

// Near-field constants; home blocks sized for about 4-8 home points each (a register chunk),
// from the density the home set would have if it filled the ball the torus map allows.
Near3 near_of(const fn3_ctx *c, bool adj)
{
    Near3 nr{};
    const Plan3 &P = c->plan;
    const Geom3 &g = c->geom;
    const double eg = P.eps_I * P.G;
    nr.e2g = eg * eg;
    nr.inv_e2g = 1.0 / nr.e2g;
    for (int k = 0; k < MAXP; ++k) nr.a[k] = P.a[k];
    for (int k = 0; k + 1 < MAXP; ++k) nr.da[k] = (k + 1) * P.a[k + 1];
    nr.cphi = P.G * INV_4PI;
    nr.cD = 2.0 / (nr.e2g * P.G);
    nr.G2 = (double)P.G * P.G;
    nr.p = P.p;
    nr.R = g.rnear;
    nr.s = g.s;
    const double dia = (0.5 - P.eps_B) * P.G;
    const double ppc = (double)(adj ? g.ns : g.nt) / std::max(1.0, PI / 6.0 * dia * dia * dia);
    static const int shapes[5][3] = {{2, 2, 1}, {2, 2, 2}, {4, 2, 2}, {4, 4, 2}, {8, 4, 2}};
    int k = 0;
    // about 4 home points per block in the forward kernel (one register chunk of 4),
    // about 8 or more in the adjoint (chunks of 8; measured on the ball lattice)
    const double want = adj ? 8.0 : 4.0;
    while (k < 4 && ppc * shapes[k][0] * shapes[k][1] * shapes[k][2] < want) ++k;
    for (int d = 0; d < 3; ++d) {
        nr.hb[d] = shapes[k][d];
        const int nb = g.ext[d] - 2 * P.m + 1;
        nr.nh[d] = (nb + nr.hb[d] - 1) / nr.hb[d];
    }
    return nr;
}

template <bool ADJ, int P>
void near3_go(fn3_ctx *c, const Near3 &nr, int nblk, size_t lds, double *phi, double *H, double *u)
{
    Buf3 &B = c->buf;
    const Geom3 &g = c->geom;
    const Map3 mp = map_of(c);
    if (!ADJ)
        k3_near<false, P><<<nblk, NB, lds, c->stream>>>(B.pos[0], B.cstart[0], B.perm[0], g.nt, B.pos[1], B.cstart[1],
                                                         B.val, g.ns, mp, nr, B.far, nullptr, phi, H);
    else
        k3_near<true, P><<<nblk, NB, lds, c->stream>>>(B.pos[1], B.cstart[1], B.perm[1], g.ns, B.pos[0], B.cstart[0],
                                                        B.aval, g.nt, mp, nr, B.far, B.w, u, nullptr);
}

template <bool ADJ>
void near3_dispatch(fn3_ctx *c, const Near3 &nr, int nblk, size_t lds, double *phi, double *H, double *u)
{
    switch (nr.p) {
    case 1: near3_go<ADJ, 1>(c, nr, nblk, lds, phi, H, u); break;
    case 2: near3_go<ADJ, 2>(c, nr, nblk, lds, phi, H, u); break;
    case 3: near3_go<ADJ, 3>(c, nr, nblk, lds, phi, H, u); break;
    case 4: near3_go<ADJ, 4>(c, nr, nblk, lds, phi, H, u); break;
    case 5: near3_go<ADJ, 5>(c, nr, nblk, lds, phi, H, u); break;
    case 6: near3_go<ADJ, 6>(c, nr, nblk, lds, phi, H, u); break;
    case 7: near3_go<ADJ, 7>(c, nr, nblk, lds, phi, H, u); break;
    case 8: near3_go<ADJ, 8>(c, nr, nblk, lds, phi, H, u); break;
    case 9: near3_go<ADJ, 9>(c, nr, nblk, lds, phi, H, u); break;
    case 10: near3_go<ADJ, 10>(c, nr, nblk, lds, phi, H, u); break;
    case 11: near3_go<ADJ, 11>(c, nr, nblk, lds, phi, H, u); break;
    default: near3_go<ADJ, 12>(c, nr, nblk, lds, phi, H, u); break;
    }
}

// the near field and the final sums of one direction
int launch_near3(fn3_ctx *c, bool adj, double *phi, double *H, double *u)
{
    const Near3 nr = near_of(c, adj);
    const int64_t nblk = (int64_t)nr.nh[0] * nr.nh[1] * nr.nh[2];
    const int nrows = (nr.hb[2] + 2 * nr.R) * (nr.hb[1] + 2 * nr.R);
    const size_t lds = near3_lds_bytes(nrows);
    if (nblk <= 0 || nblk > INT32_MAX || lds > 65536 || nr.hb[1] * nr.hb[2] > 8)
        F3_ERR(c, FN_E_DEVICE, "internal: near-field launch shape");
    if (adj) near3_dispatch<true>(c, nr, (int)nblk, lds, phi, H, u);
    else near3_dispatch<false>(c, nr, (int)nblk, lds, phi, H, u);
    F3_LAUNCH(c);
    return FN_OK;
}

int check_dev(fn3_ctx *c)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) F3_ERR(c, FN_E_DEVICE, std::string("pending HIP error: ") + hipGetErrorString(e));
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != c->device)
        if (hipSetDevice(c->device) != hipSuccess) F3_ERR(c, FN_E_DEVICE, "cannot select the context's device");
    return FN_OK;
}

// Far values of point set `set` (N points) from grid A (and B: the forward's four fields):
// by tiles when the footprints fit GATHER_TILE_LDS, else one group of lanes per point.
void launch_gather3(fn3_ctx *c, int set, int64_t N, const double2 *A, const double2 *B, double *out)
{
    const Plan3 &P = c->plan;
    Buf3 &buf = c->buf;
    const Map3 mp = map_of(c);
    const int M2 = 2 * P.m, nout = B ? 4 : 1;
    const size_t lds = gather_tile_lds(P.m, B ? 2 : 1);
    hipStream_t st = c->stream;
    if (lds <= (size_t)GATHER_TILE_LDS) {
        int nt[3];
        for (int d = 0; d < 3; ++d) nt[d] = (mp.ext[d] - M2 + 1 + ST - 1) / ST;
        const int ntiles = nt[0] * nt[1] * nt[2];
        if (M2 <= 8) {
            if (B) k3_gather_tile<8, 4><<<ntiles, 256, lds, st>>>(buf.taps[set], buf.key[set], buf.cstart[set], N, mp, nt[0], nt[1], A, B, P.G, out);
            else k3_gather_tile<8, 1><<<ntiles, 256, lds, st>>>(buf.taps[set], buf.key[set], buf.cstart[set], N, mp, nt[0], nt[1], A, B, P.G, out);
        } else {
            if (B) k3_gather_tile<16, 4><<<ntiles, 256, lds, st>>>(buf.taps[set], buf.key[set], buf.cstart[set], N, mp, nt[0], nt[1], A, B, P.G, out);
            else k3_gather_tile<16, 1><<<ntiles, 256, lds, st>>>(buf.taps[set], buf.key[set], buf.cstart[set], N, mp, nt[0], nt[1], A, B, P.G, out);
        }
    } else if (M2 <= 8) {
        k3_gather<8><<<nbk(8 * N), NT, 0, st>>>(buf.taps[set], buf.key[set], N, mp, A, B, nout, P.G, out);
    } else {
        k3_gather<16><<<nbk(16 * N), NT, 0, st>>>(buf.taps[set], buf.key[set], N, mp, A, B, nout, P.G, out);
    }
}

// spread nf value fields of set `set` (val [f][N]) over the data window, two real fields per
// complex grid (field f into grid f / 2, real part for even f, imaginary for odd f; stage
// st_spread), then transform each grid (stage st_fft)
int spread_fft(fn3_ctx *c, int set, const double *val, int64_t N, int nf, int st_spread, int st_fft)
{
    const Plan3 &P = c->plan;
    Buf3 &B = c->buf;
    const Map3 mp = map_of(c);
    const int M2 = 2 * P.m, F = ST + M2 - 1;
    int nt[3];
    for (int d = 0; d < 3; ++d) nt[d] = (mp.ext[d] - M2 + 1 + ST - 1) / ST;
    const int ntiles = nt[0] * nt[1] * nt[2];
    const int64_t cells = (int64_t)mp.ext[0] * mp.ext[1] * mp.ext[2];
    int pi = prof3_begin(c, st_spread);
    for (int f = 0; f < nf; ++f) {
        k3_spread_tile<<<ntiles, 64 * SW, (size_t)F * F * F * sizeof(double), c->stream>>>(
            B.taps[set], B.key[set], B.cstart[set], val + (int64_t)f * N, mp, nt[0], nt[1], B.tiles);
        F3_LAUNCH(c);
        k3_fold<<<nbk(cells), NT, 0, c->stream>>>(B.tiles, mp, nt[0], nt[1], nt[2], P.G, B.grid[f / 2], f % 2);
        F3_LAUNCH(c);
    }
    prof3_end(c, pi);
    pi = prof3_begin(c, st_fft);
    for (int f = 0; f < (nf + 1) / 2; ++f) {
        int rc = fft3_fwd(c, B.grid[f]);
        if (rc) return rc;
    }
    prof3_end(c, pi);
    return FN_OK;
}

}  // namespace

extern "C" {

int fn3_create(const fn_params *params, void *stream, fn3_ctx **out)
{
    if (!out) { g_err3 = "out is NULL"; return FN_E_INVAL; }
    *out = nullptr;
    if (!params) { g_err3 = "params is NULL"; return FN_E_INVAL; }
    const fn_params &p = *params;
    const int G = p.grid;
    if (G < 16 || G > MAXG3 || (G & (G - 1))) { g_err3 = "grid must be a power of two in [16, 256]"; return FN_E_INVAL; }
    if (p.m < 2 || p.m > MAXM) { g_err3 = "m must be in [2, 8]"; return FN_E_INVAL; }
    // the data window spans cells [G/4 - m, 3G/4 + m + 1] of each axis: it must fit the grid
    if (p.m > G / 4 - 1) { g_err3 = "m must be at most grid/4 - 1"; return FN_E_INVAL; }
    if (p.p < 1 || p.p > MAXP) { g_err3 = "p must be in [1, 12]"; return FN_E_INVAL; }
    if (!(p.eps_B > 0.0) || !(p.eps_B < 0.25)) { g_err3 = "eps_B must be in (0, 1/4)"; return FN_E_INVAL; }
    if (!(p.eps_I > 0.0) || !(p.eps_I * G <= 32.0) || !(p.eps_I < 0.5 - p.eps_B)) {
        g_err3 = "eps_I must be positive, eps_I*grid <= 32 and eps_I < 1/2 - eps_B";
        return FN_E_INVAL;
    }
    if (p.precision != FN_FP64) { g_err3 = "the 3D path computes in FP64 only (precision FN_FP64)"; return FN_E_UNSUPPORTED; }
    if (p.eps_S != 0.0 || p.flags != 0) { g_err3 = "eps_S and flags must be 0 in 3D"; return FN_E_UNSUPPORTED; }
    if (p.n != 0 && (p.n % 2 || 2 * p.n < G || 4 * p.n > 3 * G)) {
        g_err3 = "n must be 0 (G/2) or even with G/2 <= n <= 3G/4";
        return FN_E_INVAL;
    }
    fn3_ctx *c = new (std::nothrow) fn3_ctx();
    if (!c) { g_err3 = "out of host memory"; return FN_E_NOMEM; }
    c->prm = p;
    c->stream = static_cast<hipStream_t>(stream);
    c->debug_checks = fn::debug_checks_from_env();
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; g_err3 = "no HIP device"; return FN_E_DEVICE; }
    std::string err;
    if (!build_plan(p, c->plan, err)) { delete c; g_err3 = err; return FN_E_INVAL; }
    *out = c;
    return FN_OK;
}

int fn3_destroy(fn3_ctx *ctx)
{
    if (ctx)
        for (auto &e : ctx->prof_ev) hipEventDestroy(e);
    delete ctx;
    return FN_OK;
}

int fn3_workspace_size(const fn3_ctx *ctx, int64_t n_tgt, int64_t n_src, size_t *bytes)
{
    if (!ctx || !bytes || n_tgt < 0 || n_src < 0 || n_tgt > (int64_t)UINT32_MAX / 2 || n_src > (int64_t)UINT32_MAX / 2)
        return FN_E_INVAL;
    *bytes = layout3(ctx->plan, n_tgt, n_src).total;
    return FN_OK;
}

int fn3_set_workspace(fn3_ctx *ctx, void *dev_ptr, size_t bytes)
{
    if (!ctx) return FN_E_INVAL;
    if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255)) F3_ERR(ctx, FN_E_INVAL, "workspace must be non-NULL and 256-byte aligned");
    ctx->ws = dev_ptr;
    ctx->ws_bytes = bytes;
    ctx->plan_ready = ctx->geom_ready = ctx->charges_ready = false;
    return FN_OK;
}

int fn3_set_geometry(fn3_ctx *ctx, int64_t n_tgt, const double *tgt_xyz, int64_t n_src, const double *src_xyz,
                     const double *src_w)
{
    if (!ctx) return FN_E_INVAL;
    fn3_ctx *c = ctx;
    if (!c->ws) F3_ERR(c, FN_E_STATE, "fn3_set_workspace must be called before fn3_set_geometry");
    if (n_tgt < 0 || n_src < 0 || n_tgt + n_src < 1 || n_tgt > (int64_t)UINT32_MAX / 2 || n_src > (int64_t)UINT32_MAX / 2)
        F3_ERR(c, FN_E_INVAL, "need n_tgt, n_src >= 0, n_tgt + n_src >= 1, both < 2^31");
    if ((n_tgt > 0 && !tgt_xyz) || (n_src > 0 && (!src_xyz || !src_w))) F3_ERR(c, FN_E_INVAL, "NULL point or weight array");
    if (stream_capturing(c->stream)) F3_ERR(c, FN_E_STATE, "fn3_set_geometry waits for the device: not during graph capture");
    int rc = check_dev(c);
    if (rc) return rc;
    c->geom_ready = c->charges_ready = false;
    const Layout3 L = layout3(c->plan, n_tgt, n_src);
    if (L.total > c->ws_bytes) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "workspace too small: %zu bytes needed, %zu given", L.total, c->ws_bytes);
        F3_ERR(c, FN_E_NOMEM, msg);
    }
    bind3(c, L);
    if (!c->plan_ready) {
        rc = build_plan3(c);
        if (rc) return rc;
    }
    Buf3 &B = c->buf;
    const Plan3 &P = c->plan;
    hipStream_t st = c->stream;
    // bounding box and non-finite inputs
    double lo[3] = {1e308, 1e308, 1e308}, hi[3] = {-1e308, -1e308, -1e308}, bad = 0.0;
    const double *pts[2] = {tgt_xyz, src_xyz};
    const int64_t cnt[2] = {n_tgt, n_src};
    double h[7 * 256];
    for (int s = 0; s < 2; ++s) {
        if (cnt[s] == 0) continue;
        const int nb = (int)std::min<int64_t>(256, (cnt[s] + NT - 1) / NT);
        k3_bbox<<<nb, NT, 0, st>>>(pts[s], cnt[s], B.red);
        F3_LAUNCH(c);
        F3_HIP(c, hipMemcpyAsync(h, B.red, sizeof(double) * 7 * nb, hipMemcpyDeviceToHost, st));
        F3_HIP(c, hipStreamSynchronize(st));
        for (int b = 0; b < nb; ++b) {
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], h[7 * b + d]);
                hi[d] = std::max(hi[d], -h[7 * b + 3 + d]);
            }
            bad += h[7 * b + 6];
        }
    }
    if (n_src > 0) {
        const int nb = (int)std::min<int64_t>(256, (n_src + NT - 1) / NT);
        k3_nonfinite<<<nb, NT, 0, st>>>(src_w, n_src, B.red);
        F3_LAUNCH(c);
        F3_HIP(c, hipMemcpyAsync(h, B.red, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
        F3_HIP(c, hipStreamSynchronize(st));
        for (int b = 0; b < nb; ++b) bad += h[b];
    }
    if (bad > 0.0) F3_ERR(c, FN_E_INVAL, "non-finite coordinate or weight");
    Geom3 g;
    g.nt = n_tgt;
    g.ns = n_src;
    for (int d = 0; d < 3; ++d) g.c[d] = 0.5 * (lo[d] + hi[d]);
    double m2 = 0.0;
    for (int s = 0; s < 2; ++s) {
        if (cnt[s] == 0) continue;
        const int nb = (int)std::min<int64_t>(256, (cnt[s] + NT - 1) / NT);
        k3_maxdist<<<nb, NT, 0, st>>>(pts[s], cnt[s], g.c[0], g.c[1], g.c[2], B.red);
        F3_LAUNCH(c);
        F3_HIP(c, hipMemcpyAsync(h, B.red, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
        F3_HIP(c, hipStreamSynchronize(st));
        for (int b = 0; b < nb; ++b) m2 = std::max(m2, h[b]);
    }
    const double D = 2.0 * std::sqrt(m2);
    if (!(D > 0.0) || !std::isfinite(D)) F3_ERR(c, FN_E_DOMAIN, "all points coincide");
    g.s = (0.5 - P.eps_B) / D;
    for (int d = 0; d < 3; ++d) {
        const double umin = (g.s * (lo[d] - g.c[d])) * P.G + 0.5 * P.G;
        const double umax = (g.s * (hi[d] - g.c[d])) * P.G + 0.5 * P.G;
        g.wlo[d] = (int)std::floor(umin) - P.m;
        const int whi = (int)std::floor(umax) + P.m + 2;
        g.ext[d] = whi - g.wlo[d];
        if (g.ext[d] > L.emax || g.wlo[d] < 0 || whi > P.G) F3_ERR(c, FN_E_DEVICE, "internal: data window exceeds its bound");
    }
    g.rnear = (int)std::ceil(P.eps_I * P.G);
    c->geom = g;
    const Map3 mp = map_of(c);
    const int64_t ncell = (int64_t)g.ext[0] * g.ext[1] * g.ext[2];
    int keybits = 1;
    while (((int64_t)1 << keybits) < ncell) ++keybits;
    const double wnorm = 1.0 / (2.0 * PI * P.i0mb * std::exp(-P.m * P.kb_b));
    for (int s = 0; s < 2; ++s) {
        const int64_t n = cnt[s];
        if (n > 0) {
            k3_prepare<<<nbk(n), NT, 0, st>>>(pts[s], n, mp, B.key[s], B.perm[s]);
            F3_LAUNCH(c);
            F3_HIP(c, fn::radix_sort(B.key[s], B.perm[s], B.skey, B.sval, B.hist, n, keybits, st));
            k3_finish<<<nbk(n), NT, 0, st>>>(pts[s], s ? src_w : nullptr, n, B.perm[s], mp, P.kb_b, wnorm, B.pos[s],
                                               B.taps[s], s ? B.w : nullptr);
            F3_LAUNCH(c);
        }
        F3_HIP(c, fn::launch_cellstart(B.key[s], n, ncell, B.cstart[s], st));
        if (c->debug_checks) {  // the sort's scratch keys serve as the permutation counters
            uint32_t bad = 0;
            uint32_t *dbad = reinterpret_cast<uint32_t *>(B.red + 1024);
            const int nb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + NT - 1) / NT));
            k3_zero32<<<nb, NT, 0, st>>>(B.skey, n);
            k3_zero32<<<1, 64, 0, st>>>(dbad, 1);
            F3_LAUNCH(c);
            if (n > 0) {
                k3_check_bins<<<nb, NT, 0, st>>>(B.key[s], B.perm[s], B.cstart[s], B.pos[s], n, g.ext[0], g.ext[1],
                                                  ncell, B.skey, dbad);
                k3_check_perm<<<nb, NT, 0, st>>>(B.skey, n, dbad);
                F3_LAUNCH(c);
            }
            F3_HIP(c, hipMemcpyAsync(&bad, dbad, sizeof(bad), hipMemcpyDeviceToHost, st));
            F3_HIP(c, hipStreamSynchronize(st));
            if (bad) {
                char msg[160];
                std::snprintf(msg, sizeof msg, "debug check: %u violations in the binning of point set %d "
                              "(keys, cell starts, positions or permutation)", bad, s);
                F3_ERR(c, FN_E_DEVICE, msg);
            }
        }
    }
    F3_HIP(c, hipStreamSynchronize(st));
    c->geom_ready = true;
    c->geom_gen++;
    return FN_OK;
}

int fn3_set_charges(fn3_ctx *ctx, const double *q)
{
    if (!ctx) return FN_E_INVAL;
    fn3_ctx *c = ctx;
    if (!c->geom_ready) F3_ERR(c, FN_E_STATE, "fn3_set_geometry must succeed before fn3_set_charges");
    if (c->geom.ns > 0 && !q) F3_ERR(c, FN_E_INVAL, "q is NULL");
    int rc = check_dev(c);
    if (rc) return rc;
    if (c->geom.ns > 0) {
        const int pi = prof3_begin(c, FN3_ST_CHARGES);
        k3_values<<<nbk(c->geom.ns), NT, 0, c->stream>>>(q, c->buf.w, c->buf.perm[1], c->geom.ns, 1, c->buf.val);
        F3_LAUNCH(c);
        prof3_end(c, pi);
    }
    c->charges_ready = true;
    return FN_OK;
}

int fn3_eval(fn3_ctx *ctx, double *phi, double *H)
{
    if (!ctx) return FN_E_INVAL;
    fn3_ctx *c = ctx;
    if (!c->charges_ready) F3_ERR(c, FN_E_STATE, "fn3_set_charges must be called before fn3_eval");
    const Geom3 &g = c->geom;
    if (g.nt > 0 && !phi && !H) F3_ERR(c, FN_E_INVAL, "both outputs are NULL");
    int rc = check_dev(c);
    if (rc) return rc;
    if (g.nt == 0) return FN_OK;
    hipStream_t st = c->stream;
    Buf3 &B = c->buf;
    const Plan3 &P = c->plan;
    if (g.ns == 0) {
        if (phi) k3_fill<<<nbk(g.nt), NT, 0, st>>>(phi, g.nt, 0.0);
        if (H) k3_fill<<<nbk(3 * g.nt), NT, 0, st>>>(H, 3 * g.nt, 0.0);
        F3_LAUNCH(c);
        return FN_OK;
    }
    rc = spread_fft(c, 1, B.val, g.ns, 1, FN3_ST_SPREAD, FN3_ST_FFT);
    if (rc) return rc;
    const int64_t cb = P.n / 2 * 2 + 1, nband = cb * cb * cb;
    int pi = prof3_begin(c, FN3_ST_MULTIPLY);
    k3_mul_fwd<<<nbk(nband), NT, 0, st>>>(B.grid[0], B.grid[1], B.grid[2], P.G, P.n / 2, B.W);
    F3_LAUNCH(c);
    prof3_end(c, pi);
    pi = prof3_begin(c, FN3_ST_IFFT);
    for (int f = 1; f <= 2; ++f) {
        rc = fft3_inv(c, B.grid[f]);
        if (rc) return rc;
    }
    prof3_end(c, pi);
    const Map3 mp = map_of(c);
    // far: phi (re T1), H_z (im T1), H_x (re T2), H_y (im T2) -> far[0..3] as phi, Hx, Hy, Hz
    double *far = B.far;  // [4][nt]: phi, H_x, H_y, H_z
    pi = prof3_begin(c, FN3_ST_GATHER);
    launch_gather3(c, 0, g.nt, B.grid[1], B.grid[2], far);
    F3_LAUNCH(c);
    prof3_end(c, pi);
    pi = prof3_begin(c, FN3_ST_NEAR);
    rc = launch_near3(c, false, phi, H, nullptr);
    if (rc) return rc;
    prof3_end(c, pi);
    return FN_OK;
}

int fn3_eval_H_adjoint(fn3_ctx *ctx, const double *V, double *u)
{
    if (!ctx) return FN_E_INVAL;
    fn3_ctx *c = ctx;
    if (!c->geom_ready) F3_ERR(c, FN_E_STATE, "fn3_set_geometry must succeed before fn3_eval_H_adjoint");
    const Geom3 &g = c->geom;
    if ((g.nt > 0 && !V) || (g.ns > 0 && !u)) F3_ERR(c, FN_E_INVAL, "NULL input or output");
    int rc = check_dev(c);
    if (rc) return rc;
    hipStream_t st = c->stream;
    Buf3 &B = c->buf;
    const Plan3 &P = c->plan;
    if (g.ns == 0) return FN_OK;
    if (g.nt == 0) {
        k3_fill<<<nbk(g.ns), NT, 0, st>>>(u, g.ns, 0.0);
        F3_LAUNCH(c);
        return FN_OK;
    }
    int pi = prof3_begin(c, FN3_ST_A_VALUES);
    k3_values<<<nbk(g.nt), NT, 0, st>>>(V, nullptr, B.perm[0], g.nt, 3, B.aval);
    F3_LAUNCH(c);
    prof3_end(c, pi);
    rc = spread_fft(c, 0, B.aval, g.nt, 3, FN3_ST_A_SPREAD, FN3_ST_A_FFT);
    if (rc) return rc;
    const int64_t cb = P.n / 2 * 2 + 1, nband = cb * cb * cb;
    // T = sum_d 2 pi i l_d W F_d into grid 2, the fields unpacked from grids 0 (F0 + i F1) and 1
    pi = prof3_begin(c, FN3_ST_A_MULTIPLY);
    k3_mul_adj_packed<<<nbk(nband), NT, 0, st>>>(B.grid[0], B.grid[1], B.grid[2], P.G, P.n / 2, B.W);
    F3_LAUNCH(c);
    prof3_end(c, pi);
    pi = prof3_begin(c, FN3_ST_A_IFFT);
    rc = fft3_inv(c, B.grid[2]);
    if (rc) return rc;
    prof3_end(c, pi);
    const Map3 mp = map_of(c);
    pi = prof3_begin(c, FN3_ST_A_GATHER);
    launch_gather3(c, 1, g.ns, B.grid[2], nullptr, B.far);
    F3_LAUNCH(c);
    prof3_end(c, pi);
    pi = prof3_begin(c, FN3_ST_A_NEAR);
    rc = launch_near3(c, true, nullptr, nullptr, u);
    if (rc) return rc;
    prof3_end(c, pi);
    return FN_OK;
}

int fn3_get_info(const fn3_ctx *ctx, int64_t *n_tgt, int64_t *n_src, double *scale, int32_t *win_ext, int32_t *near_cells)
{
    if (!ctx) return FN_E_INVAL;
    if (n_tgt) *n_tgt = ctx->geom.nt;
    if (n_src) *n_src = ctx->geom.ns;
    if (scale) *scale = ctx->geom.s;
    if (win_ext)
        for (int d = 0; d < 3; ++d) win_ext[d] = ctx->geom.ext[d];
    if (near_cells) *near_cells = ctx->geom.rnear;
    return FN_OK;
}

int fn3_set_profiling(fn3_ctx *ctx, int enable)
{
    if (!ctx) return FN_E_INVAL;
    if (enable && ctx->prof_ev.empty()) {
        ctx->prof_ev.assign(2 * PROF3_MAX, nullptr);
        ctx->prof_stage.assign(PROF3_MAX, 0);
        for (auto &e : ctx->prof_ev) {
            const hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) {
                for (auto &f : ctx->prof_ev)
                    if (f) hipEventDestroy(f);
                ctx->prof_ev.clear();
                F3_ERR(ctx, FN_E_DEVICE, std::string("hipEventCreate: ") + hipGetErrorString(r));
            }
        }
    }
    ctx->prof_on = enable != 0;
    if (enable) {
        std::memset(&ctx->prof, 0, sizeof(ctx->prof));
        ctx->prof_next = 0;
    }
    return FN_OK;
}

int fn3_get_profile(fn3_ctx *ctx, fn_profile *out)
{
    if (!ctx || !out) return FN_E_INVAL;
    if (stream_capturing(ctx->stream)) F3_ERR(ctx, FN_E_STATE, "fn3_get_profile waits for the device: not during graph capture");
    for (size_t i = 0; i < ctx->prof_next; ++i) {
        F3_HIP(ctx, hipEventSynchronize(ctx->prof_ev[2 * i + 1]));
        float ms = 0.f;
        F3_HIP(ctx, hipEventElapsedTime(&ms, ctx->prof_ev[2 * i], ctx->prof_ev[2 * i + 1]));
        ctx->prof.ms[ctx->prof_stage[i]] += ms;
        ctx->prof.count[ctx->prof_stage[i]] += 1;
    }
    ctx->prof_next = 0;
    *out = ctx->prof;
    return FN_OK;
}

int fn3_internal_device(const fn3_ctx *c) { return c->device; }
void *fn3_internal_stream(const fn3_ctx *c) { return c->stream; }
uint64_t fn3_internal_geom_gen(const fn3_ctx *c) { return c->geom_gen; }

const char *fn3_last_error(const fn3_ctx *ctx)
{
    if (!ctx) return g_err3.c_str();
    return ctx->err.c_str();
}

}  // extern "C"
