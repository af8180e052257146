// Host runtime of femnfft: parameter validation, the plan (regularized kernel,
// window transform, Fourier table), workspace layout, geometry set-up and the
// evaluation pipelines behind the C-ABI declared in include/femnfft.h.
#include "fn_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

namespace fn {

static constexpr double PI = 3.14159265358979323846264338327950288;

// I0(x) by its power series sum_k (x^2/4)^k / (k!)^2 (all terms positive; used
// for x <= 40, where 120 terms reach full FP64 precision).
double bessel_i0(double x)
{
    const double q = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 200; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

void twiddles(int N, std::vector<double> &re, std::vector<double> &im)
{
    re.resize(N);
    im.resize(N);
    for (int k = 0; k < N; ++k) {
        // angle -2 pi k / N in long double, rounded to double once
        long double a = -2.0L * (long double)PI * (long double)k / (long double)N;
        re[k] = (double)std::cos(a);
        im[k] = (double)std::sin(a);
    }
}

void staged_twiddles(int N, std::vector<double> &t)
{
    t.assign(2 * (size_t)std::max(N - 8, 1), 0.0);
    int L = 1, rem = 0;
    while ((1 << rem) < N) ++rem;
    auto put = [&](int L, int rad) {
        for (int r = 1; r < rad; ++r)
            for (int k = 0; k < L; ++k) {
                const size_t i = (size_t)(L - 8) + (size_t)(r - 1) * L + k;
                const long double a = -2.0L * (long double)PI * (long double)r * k / ((long double)L * rad);
                t[2 * i] = (double)std::cos(a);
                t[2 * i + 1] = (double)std::sin(a);
            }
    };
    while (rem >= 3) {
        if (L > 1) put(L, 8);
        L <<= 3;
        rem -= 3;
    }
    if (rem >= 1 && L > 1) put(L, 1 << rem);
}

// r^q K^{(q)}(r) for K(r) = -(1/2pi) ln r.
static double K_scaled_deriv(int q, double r)
{
    if (q == 0) return -std::log(r) / (2.0 * PI);
    double f = 1.0;
    for (int i = 2; i < q; ++i) f *= i;  // (q-1)!
    return -((q % 2 == 1) ? 1.0 : -1.0) * f / (2.0 * PI);
}

static double falling(int a, int q)
{
    if (q > a) return 0.0;
    double r = 1.0;
    for (int i = 0; i < q; ++i) r *= (double)(a - i);
    return r;
}

// Gaussian elimination with partial pivoting; returns false if singular.
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
            double f = A[r * n + c] / A[c * n + c];
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

// Inner regularization polynomial at radius eps: T_I(r) = sum_k a_k (r/eps)^{2k} with
// derivatives 0..p-1 equal to those of K at eps.
static bool inner_poly(int p, double eps, double *a)
{
    std::vector<double> A(p * p), b(p), x;
    for (int q = 0; q < p; ++q) {
        for (int k = 0; k < p; ++k) A[q * p + k] = falling(2 * k, q);
        b[q] = K_scaled_deriv(q, eps);
    }
    if (!solve(A, b, p, x)) return false;
    for (int k = 0; k < MAXP; ++k) a[k] = k < p ? x[k] : 0.0;
    return true;
}

static bool build_host_plan(const fn_params &prm, Plan &P, std::string &err)
{
    P.G = prm.grid;
    P.n = prm.n ? prm.n : prm.grid / 2;
    P.m = prm.m;
    P.p = prm.p;
    P.precision = prm.precision;
    P.eps_I = prm.eps_I;
    P.eps_B = prm.eps_B;
    P.eps_S = prm.eps_S;
    P.log2G = 0;
    while ((1 << P.log2G) < P.G) ++P.log2G;
    const double sigma = (double)P.G / P.n;
    P.kb_b = PI * (2.0 - 1.0 / sigma);
    const double mb = P.m * P.kb_b;
    const double i0mb = bessel_i0(mb);
    P.win_norm = 1.0 / (2.0 * PI * i0mb * std::exp(-mb));
    // inner polynomials: at eps_I, and at eps_S for the surface sources
    if (!inner_poly(P.p, P.eps_I, P.a) || (P.eps_S > 0.0 && !inner_poly(P.p, P.eps_S, P.aS))) {
        err = "inner regularization system is singular";
        return false;
    }
    // boundary polynomial in t = (r - rB)/eps_B of degree 2p-2: Taylor part fixed
    // by K at rB, remaining p-1 coefficients make derivatives 1..p-1 vanish at t = 1
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
            if (!solve(A, b, nu, x)) {
                err = "boundary regularization system is singular";
                return false;
            }
            for (int ki = 0; ki < nu; ++ki) P.cB[p + ki] = x[ki];
        }
    }
    // window taps as polynomials in u = 2f - 1 (interpolation at WPD + 1 Chebyshev nodes)
    {
        const int D = WPD, nn = D + 1;
        const long double b = P.kb_b, mm = P.m;
        const long double i0mbl = i0mb;
        auto psi = [&](long double t) -> long double {
            const long double z2 = mm * mm - t * t;
            if (!(z2 > 0.0L)) return 0.0L;
            const long double z = std::sqrt(z2);
            return std::sinh(b * z) / ((long double)PI * z * i0mbl);
        };
        std::vector<double> A(nn * nn), rhs(nn), x;
        std::vector<double> un(nn);
        for (int k = 0; k < nn; ++k) un[k] = std::cos(PI * (k + 0.5) / nn);
        for (int r = 0; r < nn; ++r) {
            double pw = 1.0;
            for (int k = 0; k < nn; ++k) {
                A[r * nn + k] = pw;
                pw *= un[r];
            }
        }
        for (int a = 0; a < P.m; ++a) {
            for (int r = 0; r < nn; ++r)
                rhs[r] = (double)psi(0.5L * ((long double)un[r] + 1.0L) + (long double)(P.m - 1 - a));
            if (!solve(A, rhs, nn, x)) {
                err = "window interpolation system is singular";
                return false;
            }
            for (int j = 0; j < 4; ++j) {
                P.wpoly.c[a][j] = (float)x[2 * j];          // even part
                P.wpoly.c[a][4 + j] = (float)x[2 * j + 1];  // odd part
            }
        }
    }
    {
        std::vector<double> st, re, im;
        staged_twiddles(P.G, st);
        if (P.precision == FN_FP64) {
            P.twG64 = st;
        } else {
            P.twG32.resize(st.size());
            for (size_t k = 0; k < st.size(); ++k) P.twG32[k] = (float)st[k];
        }
        twiddles(P.n, re, im);
        P.twn.resize(2 * (size_t)P.n);
        for (int k = 0; k < P.n; ++k) P.twn[2 * k] = re[k], P.twn[2 * k + 1] = im[k];
    }
    P.psihat.resize(P.n / 2 + 1);
    for (int l = 0; l <= P.n / 2; ++l) {
        const double w = 2.0 * PI * l / P.G;
        P.psihat[l] = bessel_i0(P.m * std::sqrt(P.kb_b * P.kb_b - w * w)) / i0mb;
    }
    return true;
}

// slots of the 16384-double reduction scratch
enum {
    RED_COEF = 0,      // T_I coefficients (MAXP)
    RED_CB = 16,       // T_B coefficients (<= 2 MAXP - 1)
    RED_SUMQ = 64,     // sum of s_j (+ 256 partials)
    RED_SUMV = 512,    // sum of v_i (+ 256 partials)
    RED_PART = 1024,   // bounding-box partials (8 x 256)
    RED_PSI = 4096,    // window transform, n/2 + 1 <= 3073 values (n <= 3G/4)
    RED_QPART = 8192,  // block sums of the charges (2 x 1024)
    RED_VPART = 10240  // block sums of the phi-adjoint input (1024)
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static Layout make_layout(const Plan &P, int64_t nt, int64_t ns)
{
    Layout L{};
    const size_t rs = P.precision == FN_FP64 ? 8 : 4;
    const int64_t nh = P.n / 2;
    L.emax = P.G / 2 + 2 * P.m + 4;
    L.ldS = (L.emax + 63) / 64 * 64;
    const int64_t ncell = L.emax * L.emax;
    // padded tile partial sums: the larger of the two tile edges' layouts
    int64_t ptile_cells = 0;
    for (int t = TILE_MIN; t <= TILE_MAX; t *= 2) {
        const int64_t nt1 = (L.emax + t - 1) / t, pt = t + 2 * P.m - 1;
        ptile_cells = std::max(ptile_cells, nt1 * nt1 * pt * pt);
    }
    const int64_t nmax = std::max<int64_t>(std::max(nt, ns), 1);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = align256(o + bytes);
        return r;
    };
    L.off_W = take((size_t)(nh + 1) * (nh + 1) * rs);
    L.off_W2 = P.eps_S > 0.0 ? take((size_t)(nh + 1) * (nh + 1) * rs) : L.off_W;
    L.off_tw = take((size_t)P.G * 2 * rs);
    L.off_tw64 = take((size_t)P.n * 16);
    const int64_t N[2] = {std::max<int64_t>(nt, 1), std::max<int64_t>(ns, 1)};
    for (int s = 0; s < 2; ++s) {
        L.off_key[s] = take(N[s] * 4);
        L.off_perm[s] = take(N[s] * 4);
        L.off_fr32[s] = take(N[s] * 8);
        L.off_fr64[s] = take(N[s] * 16);
        L.off_cstart[s] = take((size_t)(ncell + 1) * 4);
        L.off_csub[s] = take((size_t)(ncell * NEAR_SUB + 1) * 4);
    }
    // the surface sources share the per-point source arrays, not the cell starts
    L.off_cstart[2] = P.eps_S > 0.0 ? take((size_t)(ncell + 1) * 4) : L.off_cstart[1];
    L.off_csub[2] = P.eps_S > 0.0 ? take((size_t)(ncell * NEAR_SUB + 1) * 4) : L.off_csub[1];
    L.off_w = take(N[1] * 8);
    L.off_val = take(N[1] * rs);
    L.off_val64 = take(N[1] * 8);
    L.off_aval = take(2 * N[0] * rs);
    L.off_aval64 = take(2 * N[0] * 8);
    L.off_ptile = take((size_t)2 * ptile_cells * 8);
    L.off_grid = take((size_t)3 * ncell * rs);
    // spectra: 2 fields each for input and output; the region also hosts the
    // n x n FP64 complex scratch of the plan FFT
    size_t specb = (size_t)2 * (nh + 1) * L.ldS * 2 * rs;
    size_t need = (size_t)P.n * P.n * 16;
    if (2 * specb < need) specb = (need + 1) / 2;
    L.off_spec = take(specb);
    L.off_spec2 = take(specb);
    L.off_far = take((size_t)3 * nmax * 8);
    L.off_grid_a = take((size_t)3 * ncell * rs);
    L.off_spec_a = take(specb);
    L.off_spec2_a = take(specb);
    L.off_ptile_a = take((size_t)2 * ptile_cells * 8);
    L.off_far_a = take((size_t)nmax * 8);  // the adjoint gathers one field
    L.off_red = take(16384 * 8);  // see the RED_* slots below
    L.nblk_cap = near_blocks_bound(L.emax);  // near-field home blocks of the largest window
    L.off_blk_fs = take((size_t)L.nblk_cap * 4);
    L.off_blk_as = take((size_t)L.nblk_cap * 4);
    L.off_skey = take(nmax * 4);
    L.off_sval = take(nmax * 4);
    const int64_t nblk = (nmax + 4095) / 4096;
    L.off_hist = take((size_t)256 * nblk * 4);
    L.total = o;
    return L;
}

static void bind_buffers(fn_ctx *c)
{
    char *b = static_cast<char *>(c->ws);
    const Layout &L = c->lay;
    Buffers &B = c->buf;
    B.W = b + L.off_W;
    B.W2 = b + L.off_W2;
    B.tw = b + L.off_tw;
    B.tw64 = reinterpret_cast<double2 *>(b + L.off_tw64);
    for (int s = 0; s < 2; ++s) {
        B.key[s] = reinterpret_cast<uint32_t *>(b + L.off_key[s]);
        B.perm[s] = reinterpret_cast<uint32_t *>(b + L.off_perm[s]);
        B.fr32[s] = reinterpret_cast<float *>(b + L.off_fr32[s]);
        B.fr64[s] = reinterpret_cast<double *>(b + L.off_fr64[s]);
        B.cstart[s] = reinterpret_cast<uint32_t *>(b + L.off_cstart[s]);
        B.csub[s] = reinterpret_cast<uint32_t *>(b + L.off_csub[s]);
    }
    B.cstart[2] = reinterpret_cast<uint32_t *>(b + L.off_cstart[2]);
    B.csub[2] = reinterpret_cast<uint32_t *>(b + L.off_csub[2]);
    B.key[2] = B.key[1];
    B.perm[2] = B.perm[1];
    B.fr32[2] = B.fr32[1];
    B.fr64[2] = B.fr64[1];
    B.w = reinterpret_cast<double *>(b + L.off_w);
    B.val = b + L.off_val;
    B.val64 = reinterpret_cast<double *>(b + L.off_val64);
    B.aval = b + L.off_aval;
    B.aval64 = reinterpret_cast<double *>(b + L.off_aval64);
    B.ptile = reinterpret_cast<double *>(b + L.off_ptile);
    B.grid = b + L.off_grid;
    B.spec = b + L.off_spec;
    B.spec2 = b + L.off_spec2;
    B.far = reinterpret_cast<double *>(b + L.off_far);
    B.grid_a = b + L.off_grid_a;
    B.spec_a = b + L.off_spec_a;
    B.spec2_a = b + L.off_spec2_a;
    B.ptile_a = reinterpret_cast<double *>(b + L.off_ptile_a);
    B.far_a = reinterpret_cast<double *>(b + L.off_far_a);
    B.red = reinterpret_cast<double *>(b + L.off_red);
    B.blk_fs = reinterpret_cast<uint32_t *>(b + L.off_blk_fs);
    B.blk_as = reinterpret_cast<uint32_t *>(b + L.off_blk_as);
    B.skey = reinterpret_cast<uint32_t *>(b + L.off_skey);
    B.sval = reinterpret_cast<uint32_t *>(b + L.off_sval);
    B.hist = reinterpret_cast<uint32_t *>(b + L.off_hist);
    B.scratch64 = reinterpret_cast<double *>(b + L.off_spec);
}

// Source sets 1 and 2 split the source arrays at ns1 = ns - nsurf: keys and
// permutations at offset ns1, the [2][N] fraction arrays at 2 ns1 (so that each set
// keeps the [2][N] layout of its own size).
static void bind_source_sets(fn_ctx *c, int64_t ns, int64_t nsurf)
{
    Buffers &B = c->buf;
    const int64_t ns1 = ns - nsurf;
    B.key[2] = B.key[1] + ns1;
    B.perm[2] = B.perm[1] + ns1;
    B.fr32[2] = B.fr32[1] + 2 * ns1;
    B.fr64[2] = B.fr64[1] + 2 * ns1;
}

}  // namespace fn

using namespace fn;

static thread_local std::string g_create_err;

int ctx_hip(fn_ctx *ctx, hipError_t e)
{
    if (e == hipSuccess) return FN_OK;
    ctx->err = std::string("HIP error: ") + hipGetErrorString(e);
    return FN_E_DEVICE;
}

#define FN_SET_ERR(ctx, code, msg)         \
    do {                                   \
        (ctx)->err = (msg);                \
        return (code);                     \
    } while (0)

#define FN_HIP(ctx, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            (ctx)->err = std::string("HIP error in ") + #call + ": " + hipGetErrorString(e_);    \
            return FN_E_DEVICE;                                                                  \
        }                                                                                        \
    } while (0)

// Run `call` (a launcher returning hipError_t) as stage `st`, bracketed by events
// when profiling is on.
#define FN_STAGE(ctx, st, call)                                                                  \
    do {                                                                                         \
        const int pi_ = prof_begin(ctx, st);                                                     \
        FN_HIP(ctx, call);                                                                       \
        prof_end(ctx, pi_);                                                                      \
    } while (0)

static constexpr size_t PROF_MAX = 8192;

static int prof_begin(fn_ctx *c, int st)
{
    if (!c->prof_on || stream_capturing(c->cur)) return -1;
    if (c->prof_next >= PROF_MAX) {
        c->prof.dropped++;
        return -1;
    }
    const size_t i = c->prof_next++;
    c->prof_stage[i] = st;
    hipEventRecord(c->prof_ev[2 * i], c->cur);
    return (int)i;
}

static void prof_end(fn_ctx *c, int i)
{
    if (i >= 0) hipEventRecord(c->prof_ev[2 * i + 1], c->cur);
}

static int check_device(fn_ctx *c)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->err = std::string("pending HIP error: ") + hipGetErrorString(e);
        return FN_E_DEVICE;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != c->device) {
        if (hipSetDevice(c->device) != hipSuccess) {
            c->err = "cannot select the context's device";
            return FN_E_DEVICE;
        }
    }
    return FN_OK;
}

extern "C" {

int fn_params_default(fn_params *p, int32_t grid)
{
    if (!p) return FN_E_INVAL;
    std::memset(p, 0, sizeof(*p));
    p->grid = grid;
    p->m = 6;
    p->p = 8;
    p->precision = FN_FP32_MIXED;
    p->eps_I = grid >= 2 ? 7.0 / (grid / 2) : 0.0;
    p->eps_B = 1.0 / 16.0;
    return FN_OK;
}

int fn_params_auto(int64_t n_tgt, int64_t n_src, int32_t precision, fn_params *p)
{
    if (!p || n_tgt < 0 || n_src < 0) return FN_E_INVAL;
    // small problems (fewer than 2^22 points) take p = 9: the boundary-layer error of H
    // weighs more there.  Grid: at least 2 grid cells per point, G^2 >= 2 (n_tgt + n_src),
    // or 4 for the small problems, whose near field costs more than the larger grid's
    // spread, FFT and gather
    const int64_t npt = n_tgt + n_src;
    const bool small = npt < ((int64_t)1 << 22);
    const double want = std::sqrt((small ? 4.0 : 2.0) * (double)npt);
    int32_t G = 64;
    while (G < MAXG && G < want) G *= 2;
    fn_params_default(p, G);
    p->precision = precision;
    // oversampling 4/3 (bandwidth 3G/4): the near-field radius eps_I = c/n shrinks by 2/3 at
    // the same accuracy class, so the near pairs fall to 4/9; the Kaiser-Bessel window error
    // at m = 6 stays ~1e-11
    const int nb = G >= 128 ? 3 * G / 4 : G / 2;
    p->n = G >= 128 ? nb : 0;
    p->eps_I = 7.0 / nb;
    if (small) p->p = 9;
    return FN_OK;
}

static int validate_params(const fn_params *p, std::string &err)
{
    if (!p) { err = "params is NULL"; return FN_E_INVAL; }
    const int G = p->grid;
    if (G < 64 || G > MAXG || (G & (G - 1))) { err = "grid must be a power of two in [64, 8192]"; return FN_E_INVAL; }
    if (p->m < 2 || p->m > MAXM) { err = "m must be in [2, 8]"; return FN_E_INVAL; }
    if (p->p < 1 || p->p > MAXP) { err = "p must be in [1, 12]"; return FN_E_INVAL; }
    if (!(p->eps_B > 0.0) || !(p->eps_B < 0.25)) { err = "eps_B must be in (0, 1/4)"; return FN_E_INVAL; }
    if (!(p->eps_I > 0.0) || !(p->eps_I * G <= 32.0) || !(p->eps_I < 0.5 - p->eps_B)) {
        err = "eps_I must be positive, eps_I*grid <= 32 and eps_I < 1/2 - eps_B";
        return FN_E_INVAL;
    }
    if (p->precision != FN_FP64 && p->precision != FN_FP32_MIXED) { err = "unknown precision"; return FN_E_INVAL; }
    if (p->eps_S != 0.0 && (!(p->eps_S > 0.0) || !(p->eps_S * G <= 32.0) || !(p->eps_S < 0.5 - p->eps_B))) {
        err = "eps_S must be 0, or positive with eps_S*grid <= 32 and eps_S < 1/2 - eps_B";
        return FN_E_INVAL;
    }
    if (p->flags != 0) { err = "flags must be 0"; return FN_E_UNSUPPORTED; }
    if (p->n != 0) {
        const int n = p->n;
        const int core = (n % 3 == 0) ? n / 3 : n;
        if (n % 2 || n < G / 2 || 4 * n > 3 * G || (core & (core - 1)) || core < 32) {
            err = "n must be 0, or even with G/2 <= n <= 3G/4 and a power of two or three times one (>= 96)";
            return FN_E_INVAL;
        }
    }
    return FN_OK;
}

int fn_create(const fn_params *params, void *stream, fn_ctx **out)
{
    if (!out) { g_create_err = "out is NULL"; return FN_E_INVAL; }
    *out = nullptr;
    std::string err;
    int rc = validate_params(params, err);
    if (rc) { g_create_err = err; return rc; }
    fn_ctx *c = new (std::nothrow) fn_ctx();
    if (!c) { g_create_err = "out of host memory"; return FN_E_NOMEM; }
    c->prm = *params;
    c->stream = static_cast<hipStream_t>(stream);
    c->cur = c->stream;
    c->debug_checks = debug_checks_from_env();
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        g_create_err = "no HIP device";
        return FN_E_DEVICE;
    }
    if (!build_host_plan(*params, c->plan, err)) {
        delete c;
        g_create_err = err;
        return FN_E_INVAL;
    }
    *out = c;
    return FN_OK;
}

int fn_destroy(fn_ctx *ctx)
{
    if (ctx) {
        for (auto &e : ctx->prof_ev) hipEventDestroy(e);
        if (ctx->stream2) {
            hipStreamSynchronize(ctx->stream2);
            hipStreamDestroy(ctx->stream2);
        }
        if (ctx->ev_fork) hipEventDestroy(ctx->ev_fork);
        if (ctx->ev_join) hipEventDestroy(ctx->ev_join);
    }
    delete ctx;
    return FN_OK;
}

int fn_workspace_size(const fn_ctx *ctx, int64_t n_tgt, int64_t n_src, size_t *bytes)
{
    if (!ctx || !bytes) return FN_E_INVAL;
    if (n_tgt < 0 || n_src < 0 || n_tgt > (int64_t)UINT32_MAX / 2 || n_src > (int64_t)UINT32_MAX / 2) {
        const_cast<fn_ctx *>(ctx)->err = "point counts must be in [0, 2^31)";
        return FN_E_INVAL;
    }
    *bytes = make_layout(ctx->plan, n_tgt, n_src).total;
    return FN_OK;
}

int fn_set_workspace(fn_ctx *ctx, void *dev_ptr, size_t bytes)
{
    if (!ctx) return FN_E_INVAL;
    if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255)) FN_SET_ERR(ctx, FN_E_INVAL, "workspace must be non-NULL and 256-byte aligned");
    ctx->ws = dev_ptr;
    ctx->ws_bytes = bytes;
    ctx->plan_ready = ctx->geom_ready = ctx->charges_ready = false;
    return FN_OK;
}

static int build_device_plan(fn_ctx *c)
{
    const Plan &P = c->plan;
    Buffers &B = c->buf;
    hipStream_t st = c->stream;
    // twiddles (tabulated at fn_create)
    if (P.precision == FN_FP64)
        FN_HIP(c, hipMemcpyAsync(B.tw, P.twG64.data(), P.twG64.size() * sizeof(double), hipMemcpyHostToDevice, st));
    else
        FN_HIP(c, hipMemcpyAsync(B.tw, P.twG32.data(), P.twG32.size() * sizeof(float), hipMemcpyHostToDevice, st));
    FN_HIP(c, hipMemcpyAsync(B.tw64, P.twn.data(), P.twn.size() * sizeof(double), hipMemcpyHostToDevice, st));
    double *dcoef = c->buf.red + RED_COEF;
    double *dcB = c->buf.red + RED_CB;
    double *dpsi = c->buf.red + RED_PSI;
    FN_HIP(c, hipMemcpyAsync(dcoef, P.a, sizeof(double) * MAXP, hipMemcpyHostToDevice, st));
    FN_HIP(c, hipMemcpyAsync(dcB, P.cB.data(), sizeof(double) * P.cB.size(), hipMemcpyHostToDevice, st));
    FN_HIP(c, hipMemcpyAsync(dpsi, P.psihat.data(), sizeof(double) * P.psihat.size(), hipMemcpyHostToDevice, st));
    double2 *scr = reinterpret_cast<double2 *>(B.scratch64);
    FN_HIP(c, launch_kr_samples(scr, P.n, dcoef, P.p, P.eps_I, P.eps_B, dcB, (int)P.cB.size(), st));
    FN_HIP(c, launch_fft2d_c2c64(scr, P.n, B.tw64, st));
    FN_HIP(c, launch_make_W(scr, P.n, dpsi, P.precision, B.W, st));
    if (P.eps_S > 0.0) {  // the kernel regularized at eps_S (same boundary part)
        FN_HIP(c, hipStreamSynchronize(st));
        FN_HIP(c, hipMemcpyAsync(dcoef, P.aS, sizeof(double) * MAXP, hipMemcpyHostToDevice, st));
        FN_HIP(c, launch_kr_samples(scr, P.n, dcoef, P.p, P.eps_S, P.eps_B, dcB, (int)P.cB.size(), st));
        FN_HIP(c, launch_fft2d_c2c64(scr, P.n, B.tw64, st));
        FN_HIP(c, launch_make_W(scr, P.n, dpsi, P.precision, B.W2, st));
    }
    FN_HIP(c, hipStreamSynchronize(st));
    c->plan_ready = true;
    return FN_OK;
}

// Near-field arguments of source class cls (0: eps_I, 1: surface sources at eps_S).
static NearArgs near_args(const fn_ctx *c, int cls = 0)
{
    NearArgs na{};
    const Plan &P = c->plan;
    const double eps = cls ? P.eps_S : P.eps_I;
    const double *a = cls ? P.aS : P.a;
    const double eg = eps * P.G;
    na.eps2g = eg * eg;
    na.inv_e2 = 1.0 / na.eps2g;
    na.inv_eg = 1.0 / eg;
    na.ginv = 1.0 / P.G;
    // K(eps_I) = -(1/2pi) ln(eps_I) in torus units
    const long double k_eps = -std::log((long double)eps) / (2.0L * (long double)PI);
    for (int k = 0; k < MAXP; ++k) na.u[k] = a[k];
    na.u[0] = (double)((long double)a[0] - k_eps);
    for (int k = 0; k + 1 < MAXP; ++k) na.du[k] = (k + 1) * a[k + 1];
    for (int k = 0; k < 9; ++k) na.lc[k] = 1.0 / (2 * k + 3);
    na.ln2hi = 0.693147180559945286227;
    na.ln2lo = 2.319046813846299558e-17;
    na.offset = std::log(c->geom.s) / (2.0 * PI);
    na.czero = -(a[0] + na.offset);
    na.p = P.p;
    na.rnear = cls ? c->geom.rnear_s : c->geom.rnear;
    na.f32 = P.precision == FN_FP32_MIXED ? 1 : 0;
    na.scale = c->geom.s;
    return na;
}

static int bbox_of(fn_ctx *c, const double *xy, int64_t n, double out[4], double *nonfin)
{
    // out = (min x, min y, max x, max y)
    out[0] = out[1] = 1e308;
    out[2] = out[3] = -1e308;
    if (n == 0) return FN_OK;
    const int nblk = (int)std::min<int64_t>(256, (n + 255) / 256);
    double *part = c->buf.red + RED_PART;  // 8 * 256 doubles
    FN_HIP(c, launch_bbox(xy, n, part, nblk, c->stream));
    FN_HIP(c, launch_nonfinite(xy, 2 * n, part + 4 * 256, nblk, c->stream));
    double h[8 * 256];
    FN_HIP(c, hipMemcpyAsync(h, part, sizeof(double) * 8 * 256, hipMemcpyDeviceToHost, c->stream));
    FN_HIP(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < nblk; ++b) {
        out[0] = std::min(out[0], h[4 * b]);
        out[1] = std::min(out[1], h[4 * b + 1]);
        out[2] = std::max(out[2], -h[4 * b + 2]);
        out[3] = std::max(out[3], -h[4 * b + 3]);
        *nonfin += h[4 * 256 + 4 * b];
    }
    return FN_OK;
}

static int maxdist_of(fn_ctx *c, const double *xy, int64_t n, double cx, double cy, double *m2)
{
    if (n == 0) return FN_OK;
    const int nblk = (int)std::min<int64_t>(256, (n + 255) / 256);
    double *part = c->buf.red + RED_PART;
    FN_HIP(c, launch_maxdist(xy, n, cx, cy, part, nblk, c->stream));
    double h[4 * 256];
    FN_HIP(c, hipMemcpyAsync(h, part, sizeof(double) * 4 * nblk, hipMemcpyDeviceToHost, c->stream));
    FN_HIP(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < nblk; ++b) *m2 = std::max(*m2, h[4 * b]);
    return FN_OK;
}

static int set_geometry_impl(fn_ctx *c, int64_t n_tgt, const double *tgt_xy, int64_t n_src, const double *src_xy,
                             const double *src_w, int64_t n_surf)
{
    if (!c->ws) FN_SET_ERR(c, FN_E_STATE, "fn_set_workspace must be called before fn_set_geometry");
    if (n_tgt < 0 || n_src < 0 || n_tgt + n_src < 1 || n_tgt > (int64_t)UINT32_MAX / 2 ||
        n_src > (int64_t)UINT32_MAX / 2)
        FN_SET_ERR(c, FN_E_INVAL, "need n_tgt, n_src >= 0, n_tgt + n_src >= 1, both < 2^31");
    if ((n_tgt > 0 && !tgt_xy) || (n_src > 0 && (!src_xy || !src_w)))
        FN_SET_ERR(c, FN_E_INVAL, "NULL point or weight array");
    if (n_surf < 0 || n_surf > n_src) FN_SET_ERR(c, FN_E_INVAL, "need 0 <= n_surf <= n_src");
    if (stream_capturing(c->stream)) FN_SET_ERR(c, FN_E_STATE, "fn_set_geometry waits for the device: not allowed during graph capture");
    int rc = check_device(c);
    if (rc) return rc;
    c->geom_ready = c->charges_ready = false;
    c->mesh = nullptr;
    Layout L = make_layout(c->plan, n_tgt, n_src);
    if (L.total > c->ws_bytes) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "workspace too small: %zu bytes needed, %zu given", L.total, c->ws_bytes);
        FN_SET_ERR(c, FN_E_NOMEM, msg);
    }
    c->lay = L;
    bind_buffers(c);
    if (!c->plan_ready) {
        rc = build_device_plan(c);
        if (rc) return rc;
    }
    const Plan &P = c->plan;
    Geom g;
    g.nt = n_tgt;
    g.ns = n_src;
    double bt[4], bs[4], nonfin = 0.0;
    rc = bbox_of(c, tgt_xy, n_tgt, bt, &nonfin);
    if (rc) return rc;
    rc = bbox_of(c, src_xy, n_src, bs, &nonfin);
    if (rc) return rc;
    if (n_src > 0) {
        double wn = 0.0, dummy[4];
        (void)dummy;
        const int nblk = (int)std::min<int64_t>(256, (n_src + 255) / 256);
        FN_HIP(c, launch_nonfinite(src_w, n_src, c->buf.red + RED_PART, nblk, c->stream));
        double h[4 * 256];
        FN_HIP(c, hipMemcpyAsync(h, c->buf.red + RED_PART, sizeof(double) * 4 * nblk, hipMemcpyDeviceToHost,
                                 c->stream));
        FN_HIP(c, hipStreamSynchronize(c->stream));
        for (int b = 0; b < nblk; ++b) wn += h[4 * b];
        nonfin += wn;
    }
    if (nonfin > 0.0) FN_SET_ERR(c, FN_E_INVAL, "non-finite coordinate or weight");
    const double lo[2] = {std::min(bt[0], bs[0]), std::min(bt[1], bs[1])};
    const double hi[2] = {std::max(bt[2], bs[2]), std::max(bt[3], bs[3])};
    g.c[0] = 0.5 * (lo[0] + hi[0]);
    g.c[1] = 0.5 * (lo[1] + hi[1]);
    double m2 = 0.0;
    rc = maxdist_of(c, tgt_xy, n_tgt, g.c[0], g.c[1], &m2);
    if (rc) return rc;
    rc = maxdist_of(c, src_xy, n_src, g.c[0], g.c[1], &m2);
    if (rc) return rc;
    const double D = 2.0 * std::sqrt(m2);
    if (!(D > 0.0) || !std::isfinite(D)) FN_SET_ERR(c, FN_E_DOMAIN, "all points coincide");
    g.s = (0.5 - P.eps_B) / D;
    for (int d = 0; d < 2; ++d) {
        const double umin = (g.s * (lo[d] - g.c[d])) * P.G + 0.5 * P.G;
        const double umax = (g.s * (hi[d] - g.c[d])) * P.G + 0.5 * P.G;
        const int wlo = (int)std::floor(umin) - P.m;
        const int whi = (int)std::floor(umax) + P.m + 2;
        g.wlo[d] = wlo;
        g.ext[d] = whi - wlo;
        if (g.ext[d] > L.emax || wlo < 0 || whi > P.G)
            FN_SET_ERR(c, FN_E_DEVICE, "internal: data window exceeds its bound");
        g.ntile[d] = (g.ext[d] + P.tile - 1) / P.tile;
    }
    g.rnear = (int)std::ceil(P.eps_I * P.G);
    // a second source class only when the plan has a surface radius
    g.nsurf = P.eps_S > 0.0 ? n_surf : 0;
    g.rnear_s = P.eps_S > 0.0 ? (int)std::ceil(P.eps_S * P.G) : 0;
    const int64_t ncell = (int64_t)g.ext[0] * g.ext[1];
    int keybits = 1;
    while (((int64_t)1 << keybits) < ncell * NEAR_SUB) ++keybits;
    Buffers &B = c->buf;
    bind_source_sets(c, n_src, g.nsurf);
    const int nsets = g.nsurf > 0 ? 3 : 2;
    for (int s = 0; s < nsets; ++s) {
        const int64_t n = set_size(g, s), base = set_base(g, s);
        const double *xy = s == 0 ? tgt_xy : src_xy + 2 * base;
        if (n > 0) {
            FN_HIP(c, launch_prepare(xy, n, g.c[0], g.c[1], g.s, P.G, P.m, g.wlo[0], g.wlo[1], g.ext[0],
                                     g.ext[1], B.key[s], B.perm[s], c->stream));
            FN_HIP(c, radix_sort(B.key[s], B.perm[s], B.skey, B.sval, B.hist, n, keybits, c->stream));
            FN_HIP(c, launch_finish_points(xy, s ? src_w + base : nullptr, n, B.perm[s], g.c[0], g.c[1], g.s,
                                           P.G, B.fr32[s], B.fr64[s], s ? B.w + base : nullptr, c->stream));
        }
        FN_HIP(c, launch_cellstart_sub(B.key[s], n, ncell, B.cstart[s], B.csub[s], c->stream));
        if (c->debug_checks) {  // the sort's scratch keys serve as the permutation counters
            uint32_t bad = 0;
            uint32_t *dbad = reinterpret_cast<uint32_t *>(B.red + RED_PART);
            FN_HIP(c, launch_check_bins(B.key[s], B.perm[s], B.cstart[s], B.fr32[s], B.fr64[s], n, ncell, B.skey,
                                        dbad, c->stream));
            FN_HIP(c, hipMemcpyAsync(&bad, dbad, sizeof(bad), hipMemcpyDeviceToHost, c->stream));
            FN_HIP(c, hipStreamSynchronize(c->stream));
            if (bad) {
                char msg[160];
                std::snprintf(msg, sizeof msg, "debug check: %u violations in the binning of point set %d "
                              "(keys, cell starts, fractions or permutation)", bad, s);
                FN_SET_ERR(c, FN_E_DEVICE, msg);
            }
        }
    }
    FN_HIP(c, hipStreamSynchronize(c->stream));
    c->geom = g;
    if (nsets == 3) {  // the sparse surface class: list the near blocks it needs
        uint32_t cnt[2] = {0, 0};
        uint32_t *dcnt = reinterpret_cast<uint32_t *>(B.red + RED_PART);
        const uint32_t cap = (uint32_t)L.nblk_cap;
        FN_HIP(c, launch_block_list(c->geom, B, NEAR_SURF_FWD, 0, 2, g.rnear_s, 1, B.blk_fs, cap, dcnt, c->stream));
        FN_HIP(c, launch_block_list(c->geom, B, NEAR_SURF_ADJ, 2, 0, g.rnear_s, 0, B.blk_as, cap, dcnt + 1, c->stream));
        FN_HIP(c, hipMemcpyAsync(cnt, dcnt, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
        FN_HIP(c, hipStreamSynchronize(c->stream));
        if (cnt[0] > cap || cnt[1] > cap) {
            c->geom_ready = false;
            FN_SET_ERR(c, FN_E_DEVICE, "internal: near-field block list exceeds its capacity");
        }
        c->geom.nblk_fs = (int32_t)cnt[0];
        c->geom.nblk_as = (int32_t)cnt[1];
    }
    // per source class: (target, source) pairs closer than the class radius (the near
    // field's unit of work) and pairs at exactly the same position
    for (int s = 1; s < nsets; ++s) {
        int64_t pairs = 0, coinc = 0;
        if (n_tgt > 0 && set_size(c->geom, s) > 0) {
            NearArgs na = near_args(c, s - 1);
            double *cnt = B.far;  // one count per source of the class
            double tot = 0.0;
            FN_HIP(c, launch_near_adj(c->geom, B, na, s == 2 ? NEAR_SURF_ADJ : NearShape{32, 8, 512}, s, 2,
                                      B.red + RED_SUMV, cnt, s == 2 ? B.blk_as : nullptr,
                                      c->geom.nblk_as, c->stream));
            FN_HIP(c, launch_sum(cnt, set_size(c->geom, s), B.red + RED_SUMV, c->stream));
            FN_HIP(c, hipMemcpyAsync(&tot, B.red + RED_SUMV, sizeof(double), hipMemcpyDeviceToHost, c->stream));
            FN_HIP(c, hipStreamSynchronize(c->stream));
            pairs = (int64_t)(tot + 0.5);
            FN_HIP(c, launch_coincident_count(c->geom, B, s, cnt, c->stream));
            FN_HIP(c, launch_sum(cnt, n_tgt, B.red + RED_SUMV, c->stream));
            FN_HIP(c, hipMemcpyAsync(&tot, B.red + RED_SUMV, sizeof(double), hipMemcpyDeviceToHost, c->stream));
            FN_HIP(c, hipStreamSynchronize(c->stream));
            coinc = (int64_t)(tot + 0.5);
        }
        (s == 1 ? c->geom.near_pairs : c->geom.near_pairs_s) = pairs;
        (s == 1 ? c->geom.coincident : c->geom.coincident_s) = coinc;
    }
    c->geom_ready = true;
    return FN_OK;
}

int fn_set_geometry(fn_ctx *ctx, int64_t n_tgt, const double *tgt_xy, int64_t n_src, const double *src_xy,
                    const double *src_w)
{
    if (!ctx) return FN_E_INVAL;
    return set_geometry_impl(ctx, n_tgt, tgt_xy, n_src, src_xy, src_w, 0);
}

int fn_set_geometry_split(fn_ctx *ctx, int64_t n_tgt, const double *tgt_xy, int64_t n_src, const double *src_xy,
                          const double *src_w, int64_t n_surf)
{
    if (!ctx) return FN_E_INVAL;
    return set_geometry_impl(ctx, n_tgt, tgt_xy, n_src, src_xy, src_w, n_surf);
}

int fn_set_charges(fn_ctx *ctx, const double *q)
{
    if (!ctx) return FN_E_INVAL;
    fn_ctx *c = ctx;
    if (!c->geom_ready) FN_SET_ERR(c, FN_E_STATE, "fn_set_geometry must succeed before fn_set_charges");
    if (c->geom.ns > 0 && !q) FN_SET_ERR(c, FN_E_INVAL, "q is NULL");
    int rc = check_device(c);
    if (rc) return rc;
    c->cur = c->stream;
    if (c->geom.ns > 0) {
        // per source set: its permutation indexes its own part of q (sets 1 and 2 are
        // consecutive in q, in the sorted weights and in the sorted values)
        const Geom &g = c->geom;
        const size_t rs = c->plan.precision == FN_FP64 ? 8 : 4;
        double *part = c->buf.red + RED_QPART;
        int np = 0;
        for (int s = 1; s <= 2; ++s) {
            const int64_t n = set_size(g, s), base = set_base(g, s);
            if (n == 0) continue;
            int nb = 0;
            FN_STAGE(c, FN_ST_CHARGES,
                     launch_set_values(q + base, c->buf.w + base, c->buf.perm[s], n, 1, c->plan.precision,
                                       static_cast<char *>(c->buf.val) + base * rs, c->buf.val64 + base, part + np,
                                       &nb, c->stream));
            np += nb;
        }
        FN_STAGE(c, FN_ST_CHARGES, launch_sum_partials(part, np, c->buf.red + RED_SUMQ, c->stream));
    }
    c->charges_ready = true;
    return FN_OK;
}

static int eval_impl(fn_ctx *c, double *phi, double *H, hipStream_t st)
{
    if (!c->charges_ready) FN_SET_ERR(c, FN_E_STATE, "fn_set_charges must be called before evaluation");
    if (!phi && !H && c->geom.nt > 0) FN_SET_ERR(c, FN_E_INVAL, "both outputs are NULL");
    int rc = check_device(c);
    if (rc) return rc;
    const Plan &P = c->plan;
    const Geom &g = c->geom;
    const Buffers &B = c->buf;
    c->cur = st;
    if (g.nt == 0) return FN_OK;
    if (g.ns == 0) {
        if (phi) FN_HIP(c, launch_fill(phi, g.nt, 0.0, st));
        if (H) FN_HIP(c, launch_fill(H, 2 * g.nt, 0.0, st));
        return FN_OK;
    }
    const int want_phi = phi != nullptr, want_h = H != nullptr;
    const int prec = P.precision;
    const size_t rs = prec == FN_FP64 ? 8 : 4;
    const int64_t fstride = (int64_t)g.ext[0] * g.ext[1];
    const int64_t ldS = c->lay.ldS;
    const int nh = P.n / 2;
    const int64_t sfstride = (int64_t)(nh + 1) * ldS;
    (void)rs;
    // with surface sources the two classes are spread as two fields and meet in the
    // column pass, each times its own multiplier table: sum_k W_k F_k
    const int ncls = g.nsurf > 0 ? 2 : 1;
    const size_t tfield = (size_t)g.ntile[0] * g.ntile[1] * (P.tile + 2 * P.m - 1) * (P.tile + 2 * P.m - 1);
    const char *val_s = static_cast<const char *>(B.val) + set_base(g, 2) * rs;
    FN_STAGE(c, FN_ST_SPREAD, launch_spread(prec, P, g, 1, B, B.val, 1, B.ptile, st));
    if (ncls == 2) FN_STAGE(c, FN_ST_SPREAD, launch_spread(prec, P, g, 2, B, val_s, 1, B.ptile + tfield, st));
    FN_STAGE(c, FN_ST_FOLD, launch_fold(prec, g, P.m, P.tile, B.ptile, ncls, B.grid, fstride, st));
    FN_STAGE(c, FN_ST_ROWS_FWD, launch_rows_fwd(prec, P.G, nh, B.grid, fstride, g.ext[0], g.ext[1], ncls, B.spec,
                                                ldS, B.tw, st));
    FN_STAGE(c, FN_ST_COLS, launch_cols(prec, P.G, nh, B.spec, B.spec2, sfstride, ldS, g.ext[1], COL_FWD,
                                        ncls, want_h, B.W, B.W2, B.tw, st));
    FN_STAGE(c, FN_ST_ROWS_INV, launch_rows_inv(prec, P.G, nh, B.spec2, sfstride, ldS, B.grid, fstride, g.ext[0],
                                                g.ext[1], 1, want_phi, want_h, 1, B.tw, st));
    FN_STAGE(c, FN_ST_GATHER, launch_gather(prec, P, g, 0, B, B.grid, want_h ? 3 : 1, fstride, B.far, g.nt, st));
    for (int k = 0; k < ncls; ++k) {
        const int set = 1 + k;
        if (set_size(g, set) == 0 && k > 0) continue;
        NearArgs na = near_args(c, k);
        const int stg = k ? FN_ST_NEAR_SURF : FN_ST_NEAR;
        FN_STAGE(c, stg, launch_near_fwd(g, B, na, k ? NEAR_SURF_FWD : P.near_fwd, set, k > 0, B.red + RED_SUMQ,
                                         want_phi, want_h, phi, H,
                                         k ? B.blk_fs : nullptr, g.nblk_fs, st));
        if (want_phi && (k ? g.coincident_s : g.coincident) > 0)
            FN_STAGE(c, stg, launch_near_coincident(g, B, na, 0, set, phi, st));
    }
    return FN_OK;
}

int fn_eval(fn_ctx *ctx, double *phi, double *H)
{
    if (!ctx) return FN_E_INVAL;
    return eval_impl(ctx, phi, H, ctx->stream);
}

int fn_eval_phi(fn_ctx *ctx, double *phi)
{
    if (!ctx) return FN_E_INVAL;
    if (!phi && ctx->geom.nt > 0) FN_SET_ERR(ctx, FN_E_INVAL, "phi is NULL");
    return eval_impl(ctx, phi, nullptr, ctx->stream);
}

int fn_eval_H(fn_ctx *ctx, double *H)
{
    if (!ctx) return FN_E_INVAL;
    if (!H && ctx->geom.nt > 0) FN_SET_ERR(ctx, FN_E_INVAL, "H is NULL");
    return eval_impl(ctx, nullptr, H, ctx->stream);
}

static int adjoint_impl(fn_ctx *c, const double *in, double *u, int kind, hipStream_t st)
{
    if (!c->geom_ready) FN_SET_ERR(c, FN_E_STATE, "fn_set_geometry must succeed before an adjoint evaluation");
    const Plan &P = c->plan;
    const Geom &g = c->geom;
    if ((g.nt > 0 && !in) || (g.ns > 0 && !u)) FN_SET_ERR(c, FN_E_INVAL, "NULL input or output");
    int rc = check_device(c);
    if (rc) return rc;
    // the adjoint runs on its own far-field scratch
    Buffers B = c->buf;
    B.grid = B.grid_a;
    B.spec = B.spec_a;
    B.spec2 = B.spec2_a;
    B.ptile = B.ptile_a;
    B.far = B.far_a;
    c->cur = st;
    if (g.ns == 0) return FN_OK;
    if (g.nt == 0) {
        FN_HIP(c, launch_fill(u, g.ns, 0.0, st));
        return FN_OK;
    }
    const int prec = P.precision;
    const int64_t fstride = (int64_t)g.ext[0] * g.ext[1];
    const int64_t ldS = c->lay.ldS;
    const int nh = P.n / 2;
    const int64_t sfstride = (int64_t)(nh + 1) * ldS;
    const int nf = kind == 0 ? 2 : 1;
    // with surface sources the column pass makes one spectrum per class (W_k times the
    // common input), each class gathers from its own grid
    const int ncls = g.nsurf > 0 ? 2 : 1;
    int nbv = 0;
    FN_STAGE(c, FN_ST_A_VALUES, launch_set_values(in, nullptr, B.perm[0], g.nt, nf, prec, B.aval, B.aval64,
                                                  kind == 1 ? B.red + RED_VPART : nullptr, &nbv, st));
    if (kind == 1) FN_STAGE(c, FN_ST_A_VALUES, launch_sum_partials(B.red + RED_VPART, nbv, B.red + RED_SUMV, st));
    FN_STAGE(c, FN_ST_A_SPREAD, launch_spread(prec, P, g, 0, B, B.aval, nf, B.ptile, st));
    FN_STAGE(c, FN_ST_A_FOLD, launch_fold(prec, g, P.m, P.tile, B.ptile, nf, B.grid, fstride, st));
    FN_STAGE(c, FN_ST_A_ROWS_FWD,
             launch_rows_fwd(prec, P.G, nh, B.grid, fstride, g.ext[0], g.ext[1], nf, B.spec, ldS, B.tw, st));
    FN_STAGE(c, FN_ST_A_COLS, launch_cols(prec, P.G, nh, B.spec, B.spec2, sfstride, ldS, g.ext[1],
                                          kind == 0 ? COL_ADJ_H : COL_ADJ_PHI, ncls, 0, B.W, B.W2, B.tw, st));
    FN_STAGE(c, FN_ST_A_ROWS_INV, launch_rows_inv(prec, P.G, nh, B.spec2, sfstride, ldS, B.grid, fstride, g.ext[0],
                                                  g.ext[1], 0, 1, 0, ncls, B.tw, st));
    const size_t rs = prec == FN_FP64 ? 8 : 4;
    for (int k = 0; k < ncls; ++k) {
        const int set = 1 + k;
        if (set_size(g, set) == 0) continue;
        const void *grid_k = static_cast<const char *>(B.grid) + (size_t)k * fstride * rs;
        FN_STAGE(c, FN_ST_A_GATHER, launch_gather(prec, P, g, set, B, grid_k, 1, fstride, B.far + set_base(g, set),
                                                  set_size(g, set), st));
    }
    for (int k = 0; k < ncls; ++k) {
        const int set = 1 + k;
        if (set_size(g, set) == 0) continue;
        NearArgs na = near_args(c, k);
        double *u_k = u + set_base(g, set);
        const int stg = k ? FN_ST_A_NEAR_SURF : FN_ST_A_NEAR;
        FN_STAGE(c, stg, launch_near_adj(g, B, na, k ? NEAR_SURF_ADJ : P.near_adj, set, kind, B.red + RED_SUMV, u_k,
                                         k ? B.blk_as : nullptr,
                                         g.nblk_as, st));
        if (kind == 1 && (k ? g.coincident_s : g.coincident) > 0)
            FN_STAGE(c, stg, launch_near_coincident(g, B, na, set, 0, u_k, st));
    }
    return FN_OK;
}

int fn_internal_eval_on_stream(fn_ctx *c, double *phi, double *H, hipStream_t st)
{
    const int rc = eval_impl(c, phi, H, st);
    c->cur = c->stream;
    return rc;
}

int fn_internal_adjoint_H_on_stream(fn_ctx *c, const double *V, double *u, hipStream_t st)
{
    const int rc = adjoint_impl(c, V, u, 0, st);
    c->cur = c->stream;
    return rc;
}

int fn_internal_adjoint_phi_on_stream(fn_ctx *c, const double *v, double *u, hipStream_t st)
{
    const int rc = adjoint_impl(c, v, u, 1, st);
    c->cur = c->stream;
    return rc;
}

int fn_eval_H_adjoint(fn_ctx *ctx, const double *V, double *u)
{
    if (!ctx) return FN_E_INVAL;
    return adjoint_impl(ctx, V, u, 0, ctx->stream);
}

int fn_eval_phi_adjoint(fn_ctx *ctx, const double *v, double *u)
{
    if (!ctx) return FN_E_INVAL;
    return adjoint_impl(ctx, v, u, 1, ctx->stream);
}

int fn_eval_with_H_adjoint(fn_ctx *ctx, double *phi, double *H, const double *V, double *u)
{
    if (!ctx) return FN_E_INVAL;
    fn_ctx *c = ctx;
    if (!c->charges_ready) FN_SET_ERR(c, FN_E_STATE, "fn_set_charges must be called before evaluation");
    if (!phi && !H && c->geom.nt > 0) FN_SET_ERR(c, FN_E_INVAL, "both outputs are NULL");
    if ((c->geom.nt > 0 && !V) || (c->geom.ns > 0 && !u)) FN_SET_ERR(c, FN_E_INVAL, "NULL input or output");
    int rc = check_device(c);
    if (rc) return rc;
    if (!c->stream2) {
        if (stream_capturing(c->stream))
            FN_SET_ERR(c, FN_E_STATE, "call fn_eval_with_H_adjoint once before capturing it (it creates its stream)");
        // all three or none: a failed creation leaves the context as it was
        hipStream_t s2 = nullptr;
        hipEvent_t e1 = nullptr, e2 = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&e1, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&e2, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (e2) hipEventDestroy(e2);
            if (e1) hipEventDestroy(e1);
            if (s2) hipStreamDestroy(s2);
            FN_HIP(c, e);
        }
        c->stream2 = s2;
        c->ev_fork = e1;
        c->ev_join = e2;
    }
    // fork: the adjoint on the second stream after the work already on the context's
    // stream; the forward on the context's stream; join before anything queued later
    FN_HIP(c, hipEventRecord(c->ev_fork, c->stream));
    FN_HIP(c, hipStreamWaitEvent(c->stream2, c->ev_fork, 0));
    rc = adjoint_impl(c, V, u, 0, c->stream2);
    if (rc == FN_OK) rc = eval_impl(c, phi, H, c->stream);
    // join even after an error, so that the context's stream never runs ahead of the fork
    const hipError_t e1 = hipEventRecord(c->ev_join, c->stream2);
    const hipError_t e2 = hipStreamWaitEvent(c->stream, c->ev_join, 0);
    c->cur = c->stream;
    if (rc) return rc;
    FN_HIP(c, e1);
    FN_HIP(c, e2);
    return FN_OK;
}

int fn_get_info(const fn_ctx *ctx, fn_info *info)
{
    if (!ctx || !info) return FN_E_INVAL;
    std::memset(info, 0, sizeof(*info));
    const Geom &g = ctx->geom;
    info->centre[0] = g.c[0];
    info->centre[1] = g.c[1];
    info->scale = g.s;
    info->n_tgt = g.nt;
    info->n_src = g.ns;
    for (int d = 0; d < 2; ++d) {
        info->win_lo[d] = g.wlo[d];
        info->win_ext[d] = g.ext[d];
        info->tiles[d] = g.ntile[d];
    }
    info->near_cells = g.rnear;
    info->near_pairs = g.near_pairs;
    info->n_surf = g.nsurf;
    info->near_pairs_surf = g.near_pairs_s;
    info->near_cells_surf = g.rnear_s;
    info->workspace_bytes = make_layout(ctx->plan, g.nt, g.ns).total;
    return FN_OK;
}

int fn_set_shapes(fn_ctx *ctx, const fn_shapes *shapes)
{
    if (!ctx || !shapes) return FN_E_INVAL;
    Plan &P = ctx->plan;
    const int m = P.m;
    int ng = shapes->spread_groups ? shapes->spread_groups : 0;
    if (ng < 0 || ng > 3 || (ng && 2 * ((m + ng - 1) / ng) * (2 * m) > 144))
        FN_SET_ERR(ctx, FN_E_INVAL, "spread_groups must be 0 or 1..3 with at most 144 sums per group");
    auto pick = [](int32_t bx, int32_t by, int32_t cap, const NearShape &cur) {
        NearShape s = cur;
        if (bx || by) {
            s.bx = bx;
            s.by = by;
        }
        if (cap) s.cap = cap;
        return s;
    };
    const NearShape f = pick(shapes->near_fwd_bx, shapes->near_fwd_by, shapes->near_fwd_cap, NearShape{32, 8, 1024});
    const NearShape a = pick(shapes->near_adj_bx, shapes->near_adj_by, shapes->near_adj_cap, NearShape{32, 8, 512});
    if (!near_shape_ok(f) || !near_shape_ok(a))
        FN_SET_ERR(ctx, FN_E_INVAL, "near-field shapes: 16 x 16, 32 x 8 or 64 x 4 cells, capacity a multiple of 64 in [128, 2048]");
    const int tile = shapes->tile ? shapes->tile : 32;
    if (tile != 16 && tile != 32) FN_SET_ERR(ctx, FN_E_INVAL, "tile must be 0, 16 or 32");
    P.spread_ng = ng;
    P.near_fwd = f;
    P.near_adj = a;
    P.tile = tile;
    for (int d = 0; d < 2; ++d) ctx->geom.ntile[d] = (ctx->geom.ext[d] + tile - 1) / tile;
    return FN_OK;
}

int fn_get_shapes(const fn_ctx *ctx, fn_shapes *shapes)
{
    if (!ctx || !shapes) return FN_E_INVAL;
    const Plan &P = ctx->plan;
    std::memset(shapes, 0, sizeof(*shapes));
    shapes->spread_groups = P.spread_ng ? P.spread_ng : spread_default_groups(P.m);
    shapes->near_fwd_bx = P.near_fwd.bx;
    shapes->near_fwd_by = P.near_fwd.by;
    shapes->near_fwd_cap = P.near_fwd.cap;
    shapes->near_adj_bx = P.near_adj.bx;
    shapes->near_adj_by = P.near_adj.by;
    shapes->near_adj_cap = P.near_adj.cap;
    shapes->tile = P.tile;
    return FN_OK;
}

int fn_set_profiling(fn_ctx *ctx, int enable)
{
    if (!ctx) return FN_E_INVAL;
    if (enable && ctx->prof_ev.empty()) {
        ctx->prof_ev.resize(2 * PROF_MAX);
        ctx->prof_stage.resize(PROF_MAX);
        for (auto &e : ctx->prof_ev) FN_HIP(ctx, hipEventCreate(&e));
    }
    ctx->prof_on = enable != 0;
    if (enable) {
        std::memset(&ctx->prof, 0, sizeof(ctx->prof));
        ctx->prof_next = 0;
    }
    return FN_OK;
}

int fn_get_profile(fn_ctx *ctx, fn_profile *out)
{
    if (!ctx || !out) return FN_E_INVAL;
    if (stream_capturing(ctx->stream)) FN_SET_ERR(ctx, FN_E_STATE, "fn_get_profile waits for the device: not allowed during graph capture");
    for (size_t i = 0; i < ctx->prof_next; ++i) {
        FN_HIP(ctx, hipEventSynchronize(ctx->prof_ev[2 * i + 1]));
        float ms = 0.f;
        FN_HIP(ctx, hipEventElapsedTime(&ms, ctx->prof_ev[2 * i], ctx->prof_ev[2 * i + 1]));
        ctx->prof.ms[ctx->prof_stage[i]] += ms;
        ctx->prof.count[ctx->prof_stage[i]] += 1;
    }
    ctx->prof_next = 0;
    *out = ctx->prof;
    return FN_OK;
}

const char *fn_last_error(const fn_ctx *ctx)
{
    if (!ctx) return g_create_err.c_str();
    return ctx->err.c_str();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// No-allocation evaluation: the workspace of fn_eval_noalloc is this library-owned
// device array (one copy per device, alive until the process ends).  Host code never
// passes the array's name to a kernel or a copy: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.

static __device__ __align__(256) unsigned char scratch[FN_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[NOALLOC_MAX_DEV];          // device address of `scratch` per device
bool g_noalloc_plan_ok[NOALLOC_MAX_DEV];       // the array holds the plan tables of g_noalloc_prm
fn_params g_noalloc_prm[NOALLOC_MAX_DEV];

// the device address of the scratch array on device dev (current), looked up once
int noalloc_scratch(fn_ctx *c, int dev, void **ptr)
{
    if (dev < 0 || dev >= NOALLOC_MAX_DEV) FN_SET_ERR(c, FN_E_UNSUPPORTED, "device index beyond the no-allocation table");
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            c->err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return FN_E_DEVICE;
        }
        g_noalloc_ptr[dev] = p;
    }
    *ptr = g_noalloc_ptr[dev];
    return FN_OK;
}

}  // namespace

extern "C" int fn_eval_noalloc(fn_ctx *ctx, int64_t n_tgt, const double *tgt_xy, int64_t n_src, const double *src_xy,
                               const double *src_w, int64_t n_surf, const double *q, double *phi, double *H)
{
    if (!ctx) return FN_E_INVAL;
    fn_ctx *c = ctx;
    // sizes first: nothing is read, written or launched for a problem beyond the maximum
    if (n_tgt < 0 || n_src < 0 || n_tgt + n_src < 1 || n_tgt > (int64_t)UINT32_MAX / 2 ||
        n_src > (int64_t)UINT32_MAX / 2)
        FN_SET_ERR(c, FN_E_INVAL, "need n_tgt, n_src >= 0, n_tgt + n_src >= 1, both < 2^31");
    const size_t need = make_layout(c->plan, n_tgt, n_src).total;
    if (need > (size_t)FN_NOALLOC_SCRATCH_BYTES) {
        char msg[200];
        std::snprintf(msg, sizeof msg,
                      "fn_eval_noalloc: this problem needs %zu bytes of scratch, the library's static buffer holds %zu",
                      need, (size_t)FN_NOALLOC_SCRATCH_BYTES);
        FN_SET_ERR(c, FN_E_NOMEM, msg);
    }
    if (n_src > 0 && !q) FN_SET_ERR(c, FN_E_INVAL, "q is NULL");
    if (n_tgt > 0 && !phi && !H) FN_SET_ERR(c, FN_E_INVAL, "both outputs are NULL");
    int rc = check_device(c);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    const int dev = c->device;
    void *ptr = nullptr;
    rc = noalloc_scratch(c, dev, &ptr);
    if (rc) return rc;
    // run on the static buffer, then give the context back its own workspace and state
    void *const ws0 = c->ws;
    const size_t wsb0 = c->ws_bytes;
    const bool plan0 = c->plan_ready, geom0 = c->geom_ready, charges0 = c->charges_ready;
    const Geom g0 = c->geom;
    const Layout l0 = c->lay;
    const Buffers b0 = c->buf;
    const fn_mesh *mesh0 = c->mesh;
    c->ws = ptr;
    c->ws_bytes = (size_t)FN_NOALLOC_SCRATCH_BYTES;
    // the plan tables sit at size-independent offsets: the ones the last call on this device
    // built are reused when the parameters are the same
    c->plan_ready = g_noalloc_plan_ok[dev] && std::memcmp(&g_noalloc_prm[dev], &c->prm, sizeof(fn_params)) == 0;
    g_noalloc_plan_ok[dev] = false;
    rc = set_geometry_impl(c, n_tgt, tgt_xy, n_src, src_xy, src_w, n_surf);
    if (c->plan_ready) {
        g_noalloc_prm[dev] = c->prm;
        g_noalloc_plan_ok[dev] = true;
    }
    if (rc == FN_OK) rc = fn_set_charges(c, q);
    if (rc == FN_OK) rc = eval_impl(c, phi, H, c->stream);
    c->ws = ws0;
    c->ws_bytes = wsb0;
    c->plan_ready = plan0;
    c->geom_ready = geom0;
    c->charges_ready = charges0;
    c->geom = g0;
    c->lay = l0;
    c->buf = b0;
    c->mesh = mesh0;
    return rc;
}
