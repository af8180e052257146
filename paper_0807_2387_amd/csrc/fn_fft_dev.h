// LDS line FFT building blocks shared by the 2D grid passes and the 3D path: complex
// helpers, radix-2/4/8 butterflies and a Stockham autosort pass over one line held in LDS.
// Each thread holds FFT_EPT complex values per pass; a line of N elements uses N/FFT_EPT
// threads.  Twiddles come from an FP64-generated table, never from recurrences.
#pragma once

#include "fn_internal.h"

namespace fn {
namespace fftd {

template <typename C> __device__ __forceinline__ C mk(decltype(C::x) a, decltype(C::x) b)
{
    C r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return mk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return mk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b)
{
    return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cmi(C a) { return mk<C>(a.y, -a.x); }  // a * (-i)
template <typename C> __device__ __forceinline__ C conjc(C a) { return mk<C>(a.x, -a.y); }

template <typename C> __device__ __forceinline__ void dft2(C *v)
{
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename C> __device__ __forceinline__ void dft4(C &x0, C &x1, C &x2, C &x3)
{
    C s0 = cadd(x0, x2), s1 = csub(x0, x2), s2 = cadd(x1, x3), s3 = cmi(csub(x1, x3));
    x0 = cadd(s0, s2);
    x2 = csub(s0, s2);
    x1 = cadd(s1, s3);
    x3 = csub(s1, s3);
}

template <typename C> __device__ __forceinline__ void dft4v(C *v) { dft4(v[0], v[1], v[2], v[3]); }

template <typename C> __device__ __forceinline__ void dft8(C *v)
{
    using R = decltype(C::x);
    const R h = (R)0.70710678118654752440084436210485;
    C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    // W^1 = (1 - i)/sqrt2, W^2 = -i, W^3 = (-1 - i)/sqrt2
    C t1 = mk<C>(h * (o1.x + o1.y), h * (o1.y - o1.x));
    C t2 = cmi(o2);
    C t3 = mk<C>(h * (o3.y - o3.x), -h * (o3.x + o3.y));
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, t1);
    v[5] = csub(e1, t1);
    v[2] = cadd(e2, t2);
    v[6] = csub(e2, t2);
    v[3] = cadd(e3, t3);
    v[7] = csub(e3, t3);
}

template <int RAD, typename C> __device__ __forceinline__ void dftR(C *v)
{
    if (RAD == 2) dft2(v);
    else if (RAD == 4) dft4v(v);
    else dft8(v);
}

// A line of N elements sits in LDS with one pad slot after every 8 elements:
// element i at lp(i).  Without it the first two radix-8 passes store 8 outputs
// per lane at a 64-byte lane stride (16- and 8-way bank conflicts).
__host__ __device__ constexpr int lp(int i) { return i + (i >> 3); }

// One Stockham pass over a line in LDS.  NT threads, each FFT_EPT/RAD butterflies.
// The twiddle table holds N * TWM entries (a line of a transform TWM times longer).
template <int RAD, int TWM, typename C>
__device__ __forceinline__ void fft_pass(C *buf, int N, int L, int lt, int NT, const C *__restrict__ tw)
{
    constexpr int PER = FFT_EPT / RAD;
    const int nb = N / RAD;
    C v[FFT_EPT];
#pragma unroll
    for (int c = 0; c < PER; ++c) {
        const int j = lt + c * NT;
#pragma unroll
        for (int r = 0; r < RAD; ++r) v[c * RAD + r] = buf[lp(j + r * nb)];
    }
    __syncthreads();
    const int stride = N / (L * RAD);
#pragma unroll
    for (int c = 0; c < PER; ++c) {
        const int j = lt + c * NT;
        const int k = j & (L - 1);
        if (L > 1) {
#pragma unroll
            for (int r = 1; r < RAD; ++r) v[c * RAD + r] = cmul(v[c * RAD + r], tw[r * k * stride * TWM]);
        }
        dftR<RAD>(&v[c * RAD]);
        const int o = (j - k) * RAD + k;
#pragma unroll
        for (int q = 0; q < RAD; ++q) buf[lp(o + q * L)] = v[c * RAD + q];
    }
    __syncthreads();
}

// Forward FFT of one LDS line (in place), N a power of two.  All threads of the
// block must call it.  TWM: the twiddle table belongs to a transform TWM times
// longer (entry TWM k is e^{-2 pi i k / N}).
template <int TWM = 1, typename C>
__device__ __forceinline__ void fft_line(C *buf, int N, int log2N, int lt, int NT, const C *__restrict__ tw)
{
    int L = 1, rem = log2N;
    while (rem >= 3) {
        fft_pass<8, TWM>(buf, N, L, lt, NT, tw);
        L <<= 3;
        rem -= 3;
    }
    if (rem == 2) fft_pass<4, TWM>(buf, N, L, lt, NT, tw);
    else if (rem == 1) fft_pass<2, TWM>(buf, N, L, lt, NT, tw);
}

// Pass-ordered ("staged") twiddle table of a line of N = 2^k elements, as built by
// fn::staged_twiddles on the host: the pass at sub-transform length L (> 1) and radix
// RAD keeps its (RAD - 1) L twiddles e^{-2 pi i r k / (L RAD)}, r = 1..RAD-1, k < L,
// at stw[L - 8 + (r - 1) L + k].  Radix-8 passes sit at L = 8, 64, 512, ... and the
// closing radix-4 or radix-2 pass right after the last of them, N - 8 entries in all.
// Within a pass consecutive lanes take consecutive k, so each wave's twiddle load for
// one r covers 8 consecutive entries (L = 8) or 64 (L >= 64) instead of one cache line
// per lane.
template <int RAD, typename C>
__device__ __forceinline__ void fft_pass_st(C *buf, int N, int L, int lt, int NT, const C *__restrict__ stw)
{
    constexpr int PER = FFT_EPT / RAD;
    const int nb = N / RAD;
    C v[FFT_EPT];
#pragma unroll
    for (int c = 0; c < PER; ++c) {
        const int j = lt + c * NT;
#pragma unroll
        for (int r = 0; r < RAD; ++r) v[c * RAD + r] = buf[lp(j + r * nb)];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < PER; ++c) {
        const int j = lt + c * NT;
        const int k = j & (L - 1);
        if (L > 1) {
            const C *t = stw + (L - 8) + k;
#pragma unroll
            for (int r = 1; r < RAD; ++r) v[c * RAD + r] = cmul(v[c * RAD + r], t[(r - 1) * L]);
        }
        dftR<RAD>(&v[c * RAD]);
        const int o = (j - k) * RAD + k;
#pragma unroll
        for (int q = 0; q < RAD; ++q) buf[lp(o + q * L)] = v[c * RAD + q];
    }
    __syncthreads();
}

// fft_line with a staged twiddle table of this N.
template <typename C>
__device__ __forceinline__ void fft_line_st(C *buf, int N, int log2N, int lt, int NT, const C *__restrict__ stw)
{
    int L = 1, rem = log2N;
    while (rem >= 3) {
        fft_pass_st<8>(buf, N, L, lt, NT, stw);
        L <<= 3;
        rem -= 3;
    }
    if (rem == 2) fft_pass_st<4>(buf, N, L, lt, NT, stw);
    else if (rem == 1) fft_pass_st<2>(buf, N, L, lt, NT, stw);
}

// The register-resident line FFT below needs N >= 64: then every LDS stride it uses
// (N/8 between butterfly inputs, L >= 8 between outputs) is a multiple of 8, so
// lp(j + r s) = lp(j) + r lp(s) and each access is one per-thread base plus a uniform
// offset.  opaque(lt) at the top of each pass keeps the compiler from hoisting every
// pass's addresses to the kernel entry, where they would all stay live.
__device__ __forceinline__ int opaque(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// A radix-8 pass of fft_line_reg between its first and last (8 <= L <= N / 16):
// fft_pass_st with split addresses.
template <int RAD, typename C>
__device__ __forceinline__ void fft_pass_mid(C *buf, int N, int L, int lt0, int NT, const C *__restrict__ stw)
{
    constexpr int PER = FFT_EPT / RAD;
    const int lt = opaque(lt0);
    const int snb = lp(N / RAD), sL = lp(L);
    C v[FFT_EPT];
#pragma unroll
    for (int c = 0; c < PER; ++c) {
        const C *src = buf + lp(lt + c * NT);
#pragma unroll
        for (int r = 0; r < RAD; ++r) v[c * RAD + r] = src[r * snb];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < PER; ++c) {
        const int j = lt + c * NT;
        const int k = j & (L - 1);
        const C *t = stw + (L - 8) + k;
#pragma unroll
        for (int r = 1; r < RAD; ++r) v[c * RAD + r] = cmul(v[c * RAD + r], t[(r - 1) * L]);
        dftR<RAD>(&v[c * RAD]);
        C *dst = buf + lp((j - k) * RAD + k);
#pragma unroll
        for (int q = 0; q < RAD; ++q) dst[q * sL] = v[c * RAD + q];
    }
    __syncthreads();
}

// Last pass of a line whose result stays in registers: the pass at L = N / RAD reads
// the line from LDS and leaves X[lt + i NT] in out[i] (thread lt's butterflies are
// j = lt + c NT < L, writing j + q L = lt + (c + PER q) NT).
template <int RAD, typename C>
__device__ __forceinline__ void fft_last_pass_reg(C *out, const C *buf, int N, int lt0, int NT,
                                                  const C *__restrict__ stw)
{
    constexpr int PER = FFT_EPT / RAD;
    const int lt = opaque(lt0);
    const int L = N / RAD, sL = lp(L);
    C v[FFT_EPT];
#pragma unroll
    for (int c = 0; c < PER; ++c) {
        const C *src = buf + lp(lt + c * NT);
#pragma unroll
        for (int r = 0; r < RAD; ++r) v[c * RAD + r] = src[r * sL];
    }
#pragma unroll
    for (int c = 0; c < PER; ++c) {
        const int j = lt + c * NT;
        const C *t = stw + (L - 8) + j;
#pragma unroll
        for (int r = 1; r < RAD; ++r) v[c * RAD + r] = cmul(v[c * RAD + r], t[(r - 1) * L]);
        dftR<RAD>(&v[c * RAD]);
#pragma unroll
        for (int q = 0; q < RAD; ++q) out[c + PER * q] = v[c * RAD + q];
    }
}

// Forward FFT of one line with input and output in registers: on entry v[i] holds
// x[lt + i NT], on return X[lt + i NT] (i < FFT_EPT = 8; N = 8 NT a power of two,
// N >= 64, staged twiddles of this N).  The first pass (radix 8 at L = 1, no
// twiddles) takes the registers and the last pass leaves its outputs in them, so only
// the passes in between go through the LDS line buf.  All threads of the block must
// call it; it starts with a barrier (earlier readers of buf are done), and on return
// other threads may still read buf, so barrier before writing it again.
template <typename C>
__device__ __forceinline__ void fft_line_reg(C *v, C *buf, int N, int log2N, int lt, int NT,
                                             const C *__restrict__ stw)
{
    static_assert(FFT_EPT == 8, "the first pass is one radix-8 butterfly per thread");
    dft8(v);
    __syncthreads();
    {
        C *dst = buf + 9 * opaque(lt);  // outputs 8 lt + q sit at lp(8 lt + q) = 9 lt + q
#pragma unroll
        for (int q = 0; q < 8; ++q) dst[q] = v[q];
    }
    __syncthreads();
    int L = 8, rem = log2N - 3;
    while (rem > 3) {
        fft_pass_mid<8>(buf, N, L, lt, NT, stw);
        L <<= 3;
        rem -= 3;
    }
    if (rem == 3) fft_last_pass_reg<8>(v, buf, N, lt, NT, stw);
    else if (rem == 2) fft_last_pass_reg<4>(v, buf, N, lt, NT, stw);
    else fft_last_pass_reg<2>(v, buf, N, lt, NT, stw);
}

}  // namespace fftd
}  // namespace fn
