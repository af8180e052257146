// 2D FFT passes of the fast summation, and the kernel's Fourier table.
//
// Every line transform runs in LDS as a Stockham autosort FFT (fn_fft_dev.h):
// each thread holds FFT_EPT = 8 complex values in registers per pass (one radix-8
// butterfly per pass, then a closing radix-4 or radix-2 pass), so a line of length N
// uses N/8 threads; a block of at most 1024 threads holds one line at N = 8192 and
// several shorter lines otherwise.  Twiddles come from an FP64-generated table,
// never from recurrences.  Inverse transforms are conj(FFT(conj(x))) and
// unnormalized.

// Grid layout: the real grids hold only the data window (ext_x x ext_y cells,
// row-major, x contiguous); everything outside it is zero and is supplied as
// zero padding at load time.  Because sources and targets share the window
// origin, the shift phase of the window cancels between forward and inverse
// transforms and the window can be treated as starting at index 0.
//
//   rows_fwd  : real rows -> R2C (two real lines packed in one complex FFT),
//               keep l_x in [0, n/2]; writes S[l_x][y] (y contiguous), with two
//               fields interleaved as S[l_x][y][f]
//   cols      : per l_x: FFT over y (zero-padded to G), multiply by the table
//               W(|l_x|,|l_y|) = omega b_l / (psi^(l_x/G) psi^(l_y/G))^2 on
//               |l_y| <= n/2 (zero elsewhere) and by -2 pi i l_y for H_y (or
//               the adjoint combination), inverse FFT, keep y < ext_y
//   rows_inv  : C2R of the half spectra (pairs of real outputs share one
//               complex inverse FFT); H_x = C2R((-2 pi i l_x) T_phi) needs no
//               column pass of its own because l_x is constant per column
#include "fn_fft_dev.h"

namespace fn {

namespace {

using namespace fftd;

// ---------------------------------------------------------------- plan kernels

// K_R sampled on the n x n grid (numpy FFT order), as complex FP64.
__global__ void k_kr_samples(double2 *a, int n, const double *__restrict__ coef, int p, double eps_I,
                             double eps_B, const double *__restrict__ cB, int ncB)
{
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * n) return;
    int j1 = (int)(idx / n), j2 = (int)(idx % n);
    double c1 = j1 < n / 2 ? j1 : j1 - n;
    double c2 = j2 < n / 2 ? j2 : j2 - n;
    double r = sqrt(c1 * c1 + c2 * c2) / n;
    double rB = 0.5 - eps_B, v;
    if (r < eps_I) {
        double rho2 = (r / eps_I) * (r / eps_I), acc = 0.0;
        for (int k = p - 1; k >= 0; --k) acc = acc * rho2 + coef[k];
        v = acc;
    } else if (r <= rB) {
        v = -log(r) * 0.15915494309189533576888376337251436;
    } else {
        double t = r > 0.5 ? 1.0 : (r - rB) / eps_B, acc = 0.0;
        for (int k = ncB - 1; k >= 0; --k) acc = acc * t + cB[k];
        v = acc;
    }
    a[idx] = make_double2(v, 0.0);
}

// In-place C2C forward FFT of `lines` lines of length N (a power of two, or three
// times one: r3 = 1); element e of line q at a[q * dist + e * stride]; tw holds
// the N twiddles e^{-2 pi i k/N}.  The block has exactly N/FFT_EPT threads per
// line.  For N = 3M the three decimated sequences x[3i + s] are transformed as
// M-point lines side by side, then X[j + rM] = sum_s omega^{rs} w^{sj} Y_s[j]
// (w = e^{-2 pi i/N}, omega = w^M) in place.
__global__ void __launch_bounds__(1024) k_lines64(double2 *a, int N, int log2N, int64_t stride, int64_t dist,
                                                 int lines, const double2 *__restrict__ tw, int r3)
{
    extern __shared__ double2 sh64[];
    const int NT = N / FFT_EPT, per = blockDim.x / NT;
    const int li = threadIdx.x / NT, lt = threadIdx.x % NT;
    const int q = blockIdx.x * per + li;
    double2 *buf = sh64 + (int64_t)li * lp(N);
    if (!r3) {
        for (int e = lt; e < N; e += NT) buf[lp(e)] = q < lines ? a[q * dist + e * stride] : make_double2(0, 0);
        __syncthreads();
        fft_line(buf, N, log2N, lt, NT, tw);
    } else {
        const int M = N / 3, NTs = NT / 3, grp = lt / NTs, slt = lt % NTs;
        for (int e = lt; e < N; e += NT)
            buf[lp((e % 3) * M + e / 3)] = q < lines ? a[q * dist + e * stride] : make_double2(0, 0);
        __syncthreads();
        fft_line<3>(buf + lp(grp * M), M, log2N, slt, NTs, tw);  // M is a multiple of 8
        const double c3 = -0.5, s3 = -0.86602540378443864676372317075294;  // omega = e^{-2 pi i/3}
        for (int j = lt; j < M; j += NT) {
            const double2 y0 = buf[lp(j)];
            const double2 y1 = cmul(buf[lp(M + j)], tw[j]);
            const double2 y2 = cmul(buf[lp(2 * M + j)], tw[2 * j]);
            const double2 sp = make_double2(y1.x + y2.x, y1.y + y2.y);
            const double2 sm = make_double2(y1.x - y2.x, y1.y - y2.y);
            buf[lp(j)] = make_double2(y0.x + sp.x, y0.y + sp.y);
            // y0 + c3 (y1 + y2) +- i s3 (y1 - y2)
            const double2 base = make_double2(y0.x + c3 * sp.x, y0.y + c3 * sp.y);
            buf[lp(M + j)] = make_double2(base.x - s3 * sm.y, base.y + s3 * sm.x);
            buf[lp(2 * M + j)] = make_double2(base.x + s3 * sm.y, base.y - s3 * sm.x);
        }
        __syncthreads();
    }
    if (q < lines)
        for (int e = lt; e < N; e += NT) a[q * dist + e * stride] = buf[lp(e)];
}

// W[lx * (n/2+1) + ly] = omega(lx) omega(ly) Re(b_l) / (psihat(lx) psihat(ly))^2, lx, ly in [0, n/2].
// bl holds n^2 * b_l (unnormalized DFT of the samples).
template <typename R>
__global__ void k_make_W(const double2 *__restrict__ bl, int n, const double *__restrict__ psihat, R *W)
{
    const int nh = n / 2;
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)(nh + 1) * (nh + 1)) return;
    int lx = (int)(idx / (nh + 1)), ly = (int)(idx % (nh + 1));
    double b = bl[(int64_t)(lx % n) * n + (ly % n)].x / ((double)n * n);
    double om = (lx == nh ? 0.5 : 1.0) * (ly == nh ? 0.5 : 1.0);
    double ph = psihat[lx] * psihat[ly];
    W[idx] = (R)(om * b / (ph * ph));
}

// ---------------------------------------------------------------- grid passes

// Two consecutive complex values, moved with one instruction.
template <typename C> struct alignas(2 * sizeof(C)) cpair {
    C a, b;
};

// FP32 row passes: two 1024-thread blocks (72 KB of LDS each) fit a CU when a
// thread holds at most 64 registers, which they do without spilling; the FP64
// line (147 KB) leaves room for one block only, so its registers are not capped.
#define FN_ROWS_WAVES __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 8 : 1)))

template <typename R>
__global__ void __launch_bounds__(1024) FN_ROWS_WAVES k_rows_fwd(const R *__restrict__ grid, int64_t fstride, int Ex, int Ey,
                                                  int nfield, cplx<R> *__restrict__ spec, int64_t ldS,
                                                  int G, int log2G, int nh,
                                                  const cplx<R> *__restrict__ tw)
{
    using C = cplx<R>;
    extern __shared__ char smem_rf[];
    C *sh = reinterpret_cast<C *>(smem_rf);
    const int NT = G / FFT_EPT, per = blockDim.x / NT;
    const int li = threadIdx.x / NT, lt = threadIdx.x % NT;
    const int q = xcd_block(blockIdx.x, gridDim.x) * per + li;  // spec is written transposed
    C *buf = sh + (int64_t)li * lp(G);
    // line q: nfield == 1 packs rows 2q, 2q+1; nfield == 2 packs fields 0, 1 of row q
    int ya, yb;
    const R *ra, *rb;
    if (nfield == 1) {
        ya = 2 * q;
        yb = 2 * q + 1;
        ra = ya < Ey ? grid + (int64_t)ya * Ex : nullptr;
        rb = yb < Ey ? grid + (int64_t)yb * Ex : nullptr;
    } else {
        ya = yb = q;
        ra = q < Ey ? grid + (int64_t)q * Ex : nullptr;
        rb = q < Ey ? grid + fstride + (int64_t)q * Ex : nullptr;
    }
    C v[FFT_EPT];
#pragma unroll
    for (int i = 0; i < FFT_EPT; ++i) {
        const int e = lt + i * NT;
        R a = (ra && e < Ex) ? ra[e] : (R)0;
        R b = (rb && e < Ex) ? rb[e] : (R)0;
        v[i] = mk<C>(a, b);
    }
    fft_line_reg(v, buf, G, log2G, lt, NT, tw);
    __syncthreads();  // the last pass's reads of buf are done
    {
        C *dst = buf + lp(opaque(lt));  // lp(lt + i NT) = lp(lt) + i lp(NT): NT is a multiple of 8
        const int snt = lp(NT);
#pragma unroll
        for (int i = 0; i < FFT_EPT; ++i) dst[i * snt] = v[i];
    }
    __syncthreads();
    // the transposed stores: with one field, rows 2q and 2q + 1 are neighbours in the
    // spectrum; with two, the fields are interleaved (spec[(l ldS + y) 2 + field]), so
    // either way a lane stores its two values with one 2-element store
    for (int l = lt; l <= nh; l += NT) {
        C z = buf[lp(l)], zc = conjc(buf[lp((G - l) & (G - 1))]);
        C A = mk<C>((R)0.5 * (z.x + zc.x), (R)0.5 * (z.y + zc.y));
        C B = mk<C>((R)0.5 * (z.y - zc.y), (R)-0.5 * (z.x - zc.x));
        if (nfield == 2) {
            if (ra) *reinterpret_cast<cpair<C> *>(spec + 2 * ((int64_t)l * ldS + ya)) = cpair<C>{A, B};
        } else if (rb) {
            *reinterpret_cast<cpair<C> *>(spec + (int64_t)l * ldS + ya) = cpair<C>{A, B};
        } else if (ra) {
            spec[(int64_t)l * ldS + ya] = A;
        }
    }
}

// Column pass: per l_x, the forward FFTs of the class columns, the multiply, and the
// inverse FFTs of the outputs.  The columns enter and leave through registers (thread
// lt holds y = lt + i NT), and so do the products between the forward and the inverse
// transforms: fft_line_reg keeps exactly those positions in registers.
template <typename R, int mode>
__global__ void __launch_bounds__(1024) FN_ROWS_WAVES k_cols(const cplx<R> *__restrict__ spec,
                                                             cplx<R> *__restrict__ out, int64_t ofstride,
                                                             int64_t ldS, int Ey, int nclass, int hy,
                                                             int G, int log2G, int nh, const R *__restrict__ W0,
                                                             const R *__restrict__ W1, const cplx<R> *__restrict__ tw)
{
    using C = cplx<R>;
    static_assert(FFT_EPT == 8, "fft_line_reg works on radix-8 first passes");
    extern __shared__ char smem_c[];
    C *sh = reinterpret_cast<C *>(smem_c);
    const int NT = G / FFT_EPT, per = blockDim.x / NT;
    const int li = threadIdx.x / NT, lt = threadIdx.x % NT;
    const int qx = blockIdx.x * per + li;  // l_x of this line
    const bool valid = qx <= nh;
    C *buf = sh + (int64_t)li * lp(G);
    const R twopi = (R)6.283185307179586476925286766559;
    // multiplier of class k at (qx, |l_y|); zero outside the band
    auto wmul = [&](int k, int aly) -> R {
        const R *W = k == 0 ? W0 : W1;
        return (valid && aly <= nh) ? W[(int64_t)qx * (nh + 1) + aly] : (R)0;
    };
    C acc[FFT_EPT], v[FFT_EPT];
    const int nin = mode == COL_FWD ? nclass : (mode == COL_ADJ_H ? 2 : 1);
    // two input fields come interleaved from the row pass: element y of field f at
    // spec[(qx ldS + y) 2 + f]
    const int is = nin == 2 ? 2 : 1;
#pragma unroll 1
    for (int f = 0; f < nin; ++f) {
        const C *col = spec + f + (int64_t)is * qx * ldS;
        int lt_ = opaque(lt);  // per-element indices are recomputed here, not kept live
#pragma unroll
        for (int i = 0; i < FFT_EPT; ++i) {
            const int e = lt_ + i * NT;
            v[i] = (valid && e < Ey) ? col[is * e] : mk<C>((R)0, (R)0);
        }
        fft_line_reg(v, buf, G, log2G, lt, NT, tw);
        lt_ = opaque(lt);
#pragma unroll
        for (int i = 0; i < FFT_EPT; ++i) {
            const int k = lt_ + i * NT;
            const int ly = k <= G / 2 ? k : k - G;
            const C x = v[i];
            C t;
            if (mode == COL_FWD) {
                const R w = wmul(f, ly < 0 ? -ly : ly);
                t = mk<C>(w * x.x, w * x.y);
            } else if (mode == COL_ADJ_H) {
                // (2 pi i l_d) x, l_d = l_x for component 0, l_y for component 1
                const R l = (R)(f == 0 ? qx : ly) * twopi;
                t = mk<C>(-l * x.y, l * x.x);
            } else {
                t = x;
            }
            acc[i] = (f == 0) ? t : cadd(acc[i], t);
        }
    }
    const int nout = mode == COL_FWD ? (hy ? 2 : 1) : nclass;
#pragma unroll 1
    for (int o = 0; o < nout; ++o) {
        int lt_ = opaque(lt);
#pragma unroll
        for (int i = 0; i < FFT_EPT; ++i) {
            const int k = lt_ + i * NT;
            const int ly = k <= G / 2 ? k : k - G;
            C x = acc[i];
            if (mode == COL_FWD) {
                if (o == 1) {  // (-2 pi i l_y) x
                    const R l = (R)ly * twopi;
                    x = mk<C>(l * x.y, -l * x.x);
                }
            } else {
                const R w = wmul(o, ly < 0 ? -ly : ly);
                x = mk<C>(w * x.x, w * x.y);
            }
            v[i] = conjc(x);
        }
        fft_line_reg(v, buf, G, log2G, lt, NT, tw);
        lt_ = opaque(lt);
        if (valid) {
            C *dst = out + o * ofstride + (int64_t)qx * ldS;
#pragma unroll
            for (int i = 0; i < FFT_EPT; ++i) {
                const int e = lt_ + i * NT;
                if (e < Ey) dst[e] = conjc(v[i]);
            }
        }
    }
}

// Inverse row pass.  Requested real outputs are paired into complex inverse FFTs.
// Output list entries: src (0 = T_phi/T, 1 = T_Hy), mul (0 none, 1 = -2 pi i l_x),
// dst field (0 phi, 1 Hx, 2 Hy), row offset (0 or 1).
struct OutSpec {
    int n;
    int src[6], mul[6], dst[6], dr[6];
};

template <typename R>
__global__ void __launch_bounds__(1024) FN_ROWS_WAVES k_rows_inv(const cplx<R> *__restrict__ T, int64_t tfstride, int64_t ldS,
                                                  R *__restrict__ grid, int64_t fstride, int Ex, int Ey,
                                                  OutSpec os, int G, int log2G, int nh,
                                                  const cplx<R> *__restrict__ tw)
{
    using C = cplx<R>;
    extern __shared__ char smem_ri[];
    C *sh = reinterpret_cast<C *>(smem_ri);
    const int NT = G / FFT_EPT, per = blockDim.x / NT;
    const int li = threadIdx.x / NT, lt = threadIdx.x % NT;
    const int y0 = 2 * (xcd_block(blockIdx.x, gridDim.x) * per + li);  // T is read transposed
    C *buf = sh + (int64_t)li * lp(G);
    const R twopi = (R)6.283185307179586476925286766559;
    C v[FFT_EPT];
    for (int pr = 0; pr < os.n; pr += 2) {
        const bool hasb = pr + 1 < os.n;
        const int ya = y0 + os.dr[pr], yb = hasb ? y0 + os.dr[pr + 1] : -1;
        const bool va = ya < Ey, vb = hasb && yb < Ey;
        const C *ta = T + os.src[pr] * tfstride;
        const C *tb = hasb ? T + os.src[pr + 1] * tfstride : T;
        const int ma = os.mul[pr], mb = hasb ? os.mul[pr + 1] : 0;
        // rows ya and yb = ya + 1 of one spectrum sit side by side in T (y fastest, ya even,
        // ldS a multiple of 64): one two-element load per l instead of two
        const bool adj = vb && os.src[pr + 1] == os.src[pr] && yb == ya + 1;
        int lt_ = opaque(lt);  // per-element indices are recomputed per pair, not kept live
#pragma unroll
        for (int i = 0; i < FFT_EPT; ++i) {
            const int e = lt_ + i * NT;
            C A = mk<C>((R)0, (R)0), B = mk<C>((R)0, (R)0);
            int l = -1;
            bool cj = false;
            if (e <= nh) l = e;
            else if (e >= G - nh) { l = G - e; cj = true; }
            if (l >= 0) {
                const R mlt = (R)l * twopi;
                if (adj) {
                    const cpair<C> t2 = *reinterpret_cast<const cpair<C> *>(ta + (int64_t)l * ldS + ya);
                    A = t2.a;
                    B = t2.b;
                } else {
                    if (va) A = ta[(int64_t)l * ldS + ya];
                    if (vb) B = tb[(int64_t)l * ldS + yb];
                }
                if (va) {
                    if (ma) A = mk<C>(mlt * A.y, -mlt * A.x);
                    if (l == 0) A.y = (R)0;
                    if (cj) A = conjc(A);
                }
                if (vb) {
                    if (mb) B = mk<C>(mlt * B.y, -mlt * B.x);
                    if (l == 0) B.y = (R)0;
                    if (cj) B = conjc(B);
                }
            }
            // z = A + i B, conjugated for the inverse-by-forward trick
            v[i] = mk<C>(A.x - B.y, -(A.y + B.x));
        }
        fft_line_reg(v, buf, G, log2G, lt, NT, tw);
        R *ga = grid + os.dst[pr] * fstride + (int64_t)ya * Ex;
        R *gb = grid + (hasb ? os.dst[pr + 1] : 0) * fstride + (int64_t)(hasb ? yb : 0) * Ex;
        lt_ = opaque(lt);
#pragma unroll
        for (int i = 0; i < FFT_EPT; ++i) {
            const int e = lt_ + i * NT;
            if (e < Ex) {
                const C z = v[i];  // conj of the inverse transform: real part a, imag -b
                if (va) ga[e] = z.x;
                if (vb) gb[e] = -z.y;
            }
        }
    }
}

inline int ilog2(int v)
{
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

}  // namespace

hipError_t launch_kr_samples(double2 *a, int n, const double *coef, int p, double eps_I, double eps_B,
                             const double *cB, int ncB, hipStream_t st)
{
    int64_t tot = (int64_t)n * n;
    k_kr_samples<<<(int)((tot + 255) / 256), 256, 0, st>>>(a, n, coef, p, eps_I, eps_B, cB, ncB);
    return hipGetLastError();
}

// Line FFTs of length N run on NT = N / FFT_EPT threads; a block holds enough
// lines to make at least 256 threads (one line of 1024 threads at N = 8192).
static inline int fft_nt(int N) { return N / FFT_EPT; }
static inline int fft_per(int N) { return fft_nt(N) >= 256 ? 1 : 256 / fft_nt(N); }

// n a power of two or three times one (n / FFT_EPT threads per line, at most 1024).
hipError_t launch_fft2d_c2c64(double2 *a, int n, const double2 *tw, hipStream_t st)
{
    const int r3 = (n % 3 == 0) ? 1 : 0;
    const int M = r3 ? n / 3 : n;
    if ((M & (M - 1)) || M < FFT_EPT || n / FFT_EPT > 1024) return hipErrorInvalidValue;
    const int NT = fft_nt(n);
    const int per = fft_per(n);
    const size_t lds = (size_t)per * lp(n) * sizeof(double2);
    const int lg = ilog2(M);
    int nb = (n + per - 1) / per;
    hipError_t e = hipFuncSetAttribute((const void *)k_lines64, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    k_lines64<<<nb, NT * per, lds, st>>>(a, n, lg, 1, n, n, tw, r3);  // rows
    k_lines64<<<nb, NT * per, lds, st>>>(a, n, lg, n, 1, n, tw, r3);  // columns
    return hipGetLastError();
}

hipError_t launch_make_W(const double2 *bl, int n, const double *psihat, int precision, void *W,
                         hipStream_t st)
{
    int64_t tot = (int64_t)(n / 2 + 1) * (n / 2 + 1);
    int nb = (int)((tot + 255) / 256);
    if (precision == FN_FP64) k_make_W<double><<<nb, 256, 0, st>>>(bl, n, psihat, (double *)W);
    else k_make_W<float><<<nb, 256, 0, st>>>(bl, n, psihat, (float *)W);
    return hipGetLastError();
}

template <typename R>
static size_t fft_lds_bytes(int G)
{
    return (size_t)fft_per(G) * lp(G) * sizeof(cplx<R>);
}

template <typename R>
static hipError_t rows_fwd_t(int G, int nh, const void *grid, int64_t fstride, int Ex, int Ey, int nfield,
                             void *spec, int64_t ldS, const void *tw, hipStream_t st)
{
    const int NT = fft_nt(G), per = fft_per(G);
    const int lines = (nfield == 1) ? (Ey + 1) / 2 : Ey;
    const int nb = (lines + per - 1) / per;
    hipError_t e = hipFuncSetAttribute((const void *)k_rows_fwd<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)fft_lds_bytes<R>(G));
    if (e != hipSuccess) return e;
    k_rows_fwd<R><<<nb, NT * per, fft_lds_bytes<R>(G), st>>>((const R *)grid, fstride, Ex, Ey, nfield,
                                                       (cplx<R> *)spec, ldS, G, ilog2(G), nh,
                                                       (const cplx<R> *)tw);
    return hipGetLastError();
}

hipError_t launch_rows_fwd(int precision, int G, int nh, const void *grid, int64_t fstride, int Ex, int Ey,
                           int nfield, void *spec, int64_t ldS, const void *tw,
                           hipStream_t st)
{
    if (precision == FN_FP64)
        return rows_fwd_t<double>(G, nh, grid, fstride, Ex, Ey, nfield, spec, ldS, tw, st);
    return rows_fwd_t<float>(G, nh, grid, fstride, Ex, Ey, nfield, spec, ldS, tw, st);
}

template <typename R>
static hipError_t cols_t(int G, int nh, const void *spec, void *out, int64_t ofstride,
                         int64_t ldS, int Ey, int mode, int nclass, int hy, const void *W0, const void *W1,
                         const void *tw, hipStream_t st)
{
    const int NT = fft_nt(G), per = fft_per(G);
    const int nb = (nh + 1 + per - 1) / per;
    auto kern = mode == COL_FWD ? k_cols<R, COL_FWD> : (mode == COL_ADJ_H ? k_cols<R, COL_ADJ_H> : k_cols<R, COL_ADJ_PHI>);
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)fft_lds_bytes<R>(G));
    if (e != hipSuccess) return e;
    kern<<<nb, NT * per, fft_lds_bytes<R>(G), st>>>((const cplx<R> *)spec, (cplx<R> *)out, ofstride, ldS,
                                                     Ey, nclass, hy, G, ilog2(G), nh, (const R *)W0, (const R *)W1,
                                                     (const cplx<R> *)tw);
    return hipGetLastError();
}

hipError_t launch_cols(int precision, int G, int nh, const void *spec, void *out,
                       int64_t ofstride, int64_t ldS, int Ey, int mode, int nclass, int hy, const void *W0,
                       const void *W1, const void *tw, hipStream_t st)
{
    // every table a class needs must be there: the kernel reads W1 only when nclass == 2
    if (nclass < 1 || nclass > 2 || !W0 || (nclass == 2 && !W1)) return hipErrorInvalidValue;
    if (mode != COL_FWD && mode != COL_ADJ_PHI && mode != COL_ADJ_H) return hipErrorInvalidValue;
    if (precision == FN_FP64)
        return cols_t<double>(G, nh, spec, out, ofstride, ldS, Ey, mode, nclass, hy, W0, W1, tw, st);
    return cols_t<float>(G, nh, spec, out, ofstride, ldS, Ey, mode, nclass, hy, W0, W1, tw, st);
}

template <typename R>
static hipError_t rows_inv_t(int G, int nh, const void *T, int64_t tfstride, int64_t ldS, void *grid,
                             int64_t fstride, int Ex, int Ey, int fwd, int want_phi, int want_h, int nout,
                             const void *tw, hipStream_t st)
{
    OutSpec os{};
    auto add = [&](int src, int mul, int dst, int dr) {
        os.src[os.n] = src;
        os.mul[os.n] = mul;
        os.dst[os.n] = dst;
        os.dr[os.n] = dr;
        ++os.n;
    };
    if (!fwd) {
        for (int k = 0; k < nout; ++k) {
            add(k, 0, k, 0);
            add(k, 0, k, 1);
        }
    } else {
        // a complex transform pairs the same field on two rows: fields of very
        // different magnitude (phi and H) must not share one transform, or the
        // rounding of the larger one swamps the smaller one
        if (want_phi && want_h) {
            add(0, 0, 0, 0); add(0, 0, 0, 1);   // phi_y + i phi_y+1
            add(0, 1, 1, 0); add(0, 1, 1, 1);   // Hx_y + i Hx_y+1
            add(1, 0, 2, 0); add(1, 0, 2, 1);   // Hy_y + i Hy_y+1
        } else if (want_phi) {
            add(0, 0, 0, 0); add(0, 0, 0, 1);
        } else {
            add(0, 1, 1, 0); add(0, 1, 1, 1);
            add(1, 0, 2, 0); add(1, 0, 2, 1);
        }
    }
    const int NT = fft_nt(G), per = fft_per(G);
    const int lines = (Ey + 1) / 2;
    const int nb = (lines + per - 1) / per;
    hipError_t e = hipFuncSetAttribute((const void *)k_rows_inv<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)fft_lds_bytes<R>(G));
    if (e != hipSuccess) return e;
    k_rows_inv<R><<<nb, NT * per, fft_lds_bytes<R>(G), st>>>((const cplx<R> *)T, tfstride, ldS, (R *)grid, fstride,
                                                        Ex, Ey, os, G, ilog2(G), nh, (const cplx<R> *)tw);
    return hipGetLastError();
}

hipError_t launch_rows_inv(int precision, int G, int nh, const void *T, int64_t tfstride, int64_t ldS,
                           void *grid, int64_t fstride, int Ex, int Ey, int fwd, int want_phi, int want_h,
                           int nout, const void *tw, hipStream_t st)
{
    if (nout < 1 || nout > 2) return hipErrorInvalidValue;
    if (precision == FN_FP64)
        return rows_inv_t<double>(G, nh, T, tfstride, ldS, grid, fstride, Ex, Ey, fwd, want_phi, want_h, nout,
                                  tw, st);
    return rows_inv_t<float>(G, nh, T, tfstride, ldS, grid, fstride, Ex, Ey, fwd, want_phi, want_h, nout, tw,
                             st);
}


}  // namespace fn
