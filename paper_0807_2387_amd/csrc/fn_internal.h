// Internal declarations of the femnfft library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "femnfft.h"

namespace fn {

constexpr int TILE_MIN = 16;    // spread / gather tile edges in grid cells: 16 or 32 (Plan::tile)
constexpr int TILE_MAX = 32;
constexpr int MAXM = 8;         // largest window half-width
constexpr int MAXP = 12;        // largest regularization degree
constexpr int FFT_EPT = 8;      // complex elements held per thread in the LDS FFT
constexpr int MAXG = 8192;      // largest FFT grid
// Points are sorted by cell and, inside a cell, by which of NEAR_SUB equal x slices of it
// they lie in; the near field cuts each row's candidates at those slice starts.
constexpr int NEAR_SUB_LOG2 = 2;
constexpr int NEAR_SUB = 1 << NEAR_SUB_LOG2;

// Workgroups are handed to the 8 XCDs round-robin (block b to XCD b % 8), and
// each XCD has its own L2.  xcd_block maps the i-th block of XCD x to logical
// block x * (nb / 8) + min(x, nb % 8) + i, a bijection of [0, nb), so that one
// XCD works on a contiguous range of lines and blocks sharing cache lines meet
// in one L2.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int x = b % NXCD, i = b / NXCD, q = nb / NXCD, r = nb % NXCD;
    return x * q + (x < r ? x : r) + i;
}

template <typename R> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
template <> struct cplx_t<double> { using type = double2; };
template <typename R> using cplx = typename cplx_t<R>::type;

// Host-side plan: everything that depends only on the parameters.
// The window's taps of a point with in-cell fraction f, as polynomials of degree
// WPD in u = 2f - 1 interpolated at Chebyshev nodes; used by the FP32 spread and
// gather.  The window is even, so tap 2m-1-a at u is tap a at -u: only taps
// a < m are stored, split as p_a(u) = E_a(u^2) + u O_a(u^2) with E_a's
// coefficients at c[a][0..3] and O_a's at c[a][4..7] (ascending powers of u^2).
constexpr int WPD = 7;
struct WinPoly {
    float c[MAXM][WPD + 1];
};

// Near-field work shape: home blocks of bx x by cells (bx by = 256: 16 x 16, 32 x 8 or
// 64 x 4) and the staging capacity in points per LDS chunk (a multiple of 64 in
// [128, 2048]).
struct NearShape {
    int bx = 32, by = 8, cap = 1024;
};
// the sparse surface class keeps one shape (its block lists are built at set-up)
constexpr NearShape NEAR_SURF_FWD{32, 8, 512};
constexpr NearShape NEAR_SURF_ADJ{32, 8, 1024};

struct Plan {
    int G = 0, n = 0, m = 0, p = 0, log2G = 0;
    int precision = FN_FP32_MIXED;
    double eps_I = 0, eps_B = 0;
    double eps_S = 0;                // near radius of the surface sources (0: no second class)
    WinPoly wpoly{};                 // per-tap polynomials of the window (FP32 path)
    double kb_b = 0;                 // Kaiser-Bessel shape b = pi (2 - 1/sigma)
    double win_norm = 0;             // 1 / (2 pi I0(m b) e^{-m b})
    double a[MAXP] = {0};            // inner polynomial T_I(r) = sum_k a_k (r/eps_I)^{2k}
    double aS[MAXP] = {0};           // the same at eps_S (surface sources)
    std::vector<double> cB;          // boundary polynomial in t = (r - r_B)/eps_B
    std::vector<double> psihat;      // window transform at l/G, l = 0..n/2
    int spread_ng = 0;               // row groups of the FP32 spread footprint (0: spread_default_groups)
    int tile = 32;                   // spread / gather tile edge, cells (16 or 32)
    NearShape near_fwd{32, 8, 1024}; // near-field shape of the forward volume-class kernel
    NearShape near_adj{32, 8, 512};  // ... and of the adjoint one
    // FFT twiddles computed at fn_create: the grid passes' pass-ordered table of a G-point
    // line in the grid precision (float2 or double2 pairs as consecutive values,
    // staged_twiddles), and e^{-2 pi i k/n}, k < n, in FP64 (plan transform)
    std::vector<double> twG64;       // [G - 8][2], FP64 path
    std::vector<float> twG32;        // [G - 8][2], FP32-mixed path
    std::vector<double> twn;         // [n][2]
};

// Per-geometry facts (host copy).
struct Geom {
    int64_t nt = 0, ns = 0;
    double c[2] = {0, 0};
    double s = 0;
    int32_t wlo[2] = {0, 0};
    int32_t ext[2] = {0, 0};         // window extent (cells) x, y
    int32_t ntile[2] = {0, 0};       // spread / gather tiles per dim (of the plan's tile edge)
    int32_t rnear = 0;               // near radius in cells
    int64_t near_pairs = 0;          // pairs closer than eps_I
    int64_t coincident = 0;          // (target, source) pairs at exactly the same position
    // surface sources: the last nsurf sources, near radius eps_S (nsurf > 0 only when
    // the plan has eps_S > 0); the counts above then cover the volume sources only
    int64_t nsurf = 0;
    int32_t rnear_s = 0;
    int64_t near_pairs_s = 0;
    int64_t coincident_s = 0;
    int32_t nblk_fs = 0, nblk_as = 0;  // listed near blocks of the surface class (forward, adjoint)
};

// Point sets: 0 = targets, 1 = (volume) sources, 2 = surface sources.  Sets 1 and 2
// share the source arrays: set 2 starts at source index set_base(g, 2).
inline int64_t set_size(const Geom &g, int s) { return s == 0 ? g.nt : (s == 1 ? g.ns - g.nsurf : g.nsurf); }
inline int64_t set_base(const Geom &g, int s) { return s == 2 ? g.ns - g.nsurf : 0; }

// Row groups of the FP32 spread's register footprint for window half-width m: every
// group holds whole row pairs, at most 72 FP32 sums per group by default (one group of
// 4 m^2 sums at m <= 4).
inline int spread_default_groups(int m) { return m <= 5 ? 1 : (m <= 6 ? 2 : 3); }

// Device arrays carved out of the caller's workspace.
struct Buffers {
    // plan
    void *W = nullptr;               // multiplier table [(n/2+1) x (n/2+1)], R
    void *W2 = nullptr;              // the same for the kernel regularized at eps_S
    void *tw = nullptr;              // grid-pass twiddles (staged_twiddles(G)), cplx<R>
    double2 *tw64 = nullptr;         // FP64 twiddles for the plan FFT (length n)
    // geometry, per point set (see set_size), each sorted by cell; perm[s] holds indices
    // relative to the set's first point
    uint32_t *key[3] = {nullptr, nullptr, nullptr};
    uint32_t *perm[3] = {nullptr, nullptr, nullptr};
    float *fr32[3] = {nullptr, nullptr, nullptr};   // [2][N] in-cell fractions, FP32
    double *fr64[3] = {nullptr, nullptr, nullptr};  // [2][N] in-cell fractions, FP64
    uint32_t *cstart[3] = {nullptr, nullptr, nullptr}; // [ncell + 1]
    uint32_t *csub[3] = {nullptr, nullptr, nullptr};   // [ncell NEAR_SUB + 1] starts of the x slices
    double *w = nullptr;             // source weights, sorted (set 1, then set 2)
    // per-evaluation data
    void *val = nullptr;             // charges s_j = w_j q_j, R, sorted sources (set 1, then set 2)
    double *val64 = nullptr;         // the same in FP64 (near field)
    void *aval = nullptr;            // adjoint inputs (v or V), R, [2][nt] sorted targets
    double *aval64 = nullptr;        // the same in FP64
    double *ptile = nullptr;         // padded tile partial sums, FP64, 2 fields
    void *grid = nullptr;            // real grids, R, 3 fields x ext^2 (max)
    void *spec = nullptr;            // half spectra, cplx<R>, 2 fields x (n/2+1) x ldS
    void *spec2 = nullptr;           // column-pass outputs, cplx<R>, 2 fields
    double *far = nullptr;           // [3][max(nt, ns)] far-field results, sorted order
    // the adjoint's own far-field scratch (grid, spectra, tile sums, results), so that a
    // forward and an adjoint evaluation can run at the same time (fn_eval_with_H_adjoint)
    void *grid_a = nullptr, *spec_a = nullptr, *spec2_a = nullptr;
    double *ptile_a = nullptr, *far_a = nullptr;
    double *red = nullptr;           // reduction scratch
    uint32_t *blk_fs = nullptr;      // near blocks of the surface class: targets near surface sources
    uint32_t *blk_as = nullptr;      // near blocks of the surface class: blocks holding surface sources
    // sort scratch
    uint32_t *skey = nullptr, *sval = nullptr, *hist = nullptr;
    double *scratch64 = nullptr;     // plan FFT scratch (n x n complex) aliases grid/spec
};

struct Layout {
    size_t total = 0;
    size_t off_W, off_W2, off_tw, off_tw64;
    size_t off_key[2], off_perm[2], off_fr32[2], off_fr64[2], off_cstart[3], off_csub[3];
    size_t off_w, off_val, off_val64, off_aval, off_aval64, off_ptile, off_grid, off_spec, off_spec2, off_far, off_red;
    size_t off_blk_fs, off_blk_as;
    size_t off_grid_a, off_spec_a, off_spec2_a, off_ptile_a, off_far_a;
    size_t off_skey, off_sval, off_hist;
    int64_t emax = 0;                // bound on the window extent
    int64_t nblk_cap = 0;            // capacity of the near-field block lists
    int64_t ldS = 0;                 // leading dimension of the spectra
};

}  // namespace fn

struct fn_mesh;

struct fn_ctx {
    fn_params prm{};
    fn::Plan plan;
    fn::Geom geom;
    fn::Buffers buf;
    fn::Layout lay;
    hipStream_t stream = nullptr;
    hipStream_t cur = nullptr;       // stream the pipeline being enqueued runs on (stage events)
    hipStream_t stream2 = nullptr;   // second stream of fn_eval_with_H_adjoint (created on first use)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int device = 0;
    bool debug_checks = false;       // FEMNFFT_DEBUG_CHECKS: validate the binning after set_geometry
    void *ws = nullptr;
    size_t ws_bytes = 0;
    int64_t ws_nt = 0, ws_ns = 0;    // sizes the workspace was laid out for
    // stage profiling (events recorded on the stream)
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;      // pool, 2 per stage record
    std::vector<int> prof_stage;          // stage of each recorded pair
    size_t prof_next = 0;
    fn_profile prof{};
    bool plan_ready = false;
    bool geom_ready = false;
    bool charges_ready = false;
    const fn_mesh *mesh = nullptr;   // mesh whose nodes and sources are the geometry (fn_bind_mesh)
    uint64_t mesh_stamp = 0;
    bool mesh_at_sources = false;    // fn_bind_mesh_sources: targets are the mesh's quadrature points
    std::string err;
};

// FN_OK, or FN_E_DEVICE with the HIP message stored in ctx->err
int ctx_hip(fn_ctx *ctx, hipError_t e);

// fn_eval / fn_eval_H_adjoint with their work enqueued on `st` (which must be ordered
// after the context's stream by the caller; the two directions use separate scratch).
// Library-internal (hidden from the shared object's exports).
extern "C" {
__attribute__((visibility("hidden"))) int fn_internal_eval_on_stream(fn_ctx *c, double *phi, double *H,
                                                                     hipStream_t st);
__attribute__((visibility("hidden"))) int fn_internal_adjoint_H_on_stream(fn_ctx *c, const double *V, double *u,
                                                                          hipStream_t st);
__attribute__((visibility("hidden"))) int fn_internal_adjoint_phi_on_stream(fn_ctx *c, const double *v, double *u,
                                                                            hipStream_t st);
// the 3D context's device, stream and geometry generation (incremented by every successful
// fn3_set_geometry), for the 3D FEM front
__attribute__((visibility("hidden"))) int fn3_internal_device(const fn3_ctx *c);
__attribute__((visibility("hidden"))) void *fn3_internal_stream(const fn3_ctx *c);
__attribute__((visibility("hidden"))) uint64_t fn3_internal_geom_gen(const fn3_ctx *c);
}

// true while work issued on `st` is being captured into a graph
inline bool stream_capturing(hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive;
}

namespace fn {

// ---- kernel launchers (defined in the .hip files) ----
// geometry
hipError_t launch_bbox(const double *p, int64_t n, double *part, int nblk, hipStream_t st);
hipError_t launch_maxdist(const double *p, int64_t n, double cx, double cy, double *part, int nblk,
                          hipStream_t st);
hipError_t launch_nonfinite(const double *p, int64_t n, double *part, int nblk, hipStream_t st);
hipError_t launch_prepare(const double *xy, int64_t n, double cx, double cy, double s, int G, int m,
                          int wlox, int wloy, int extx, int exty, uint32_t *key, uint32_t *idx,
                          hipStream_t st);
hipError_t radix_sort(uint32_t *key, uint32_t *val, uint32_t *key2, uint32_t *val2, uint32_t *hist,
                      int64_t n, int keybits, hipStream_t st);  // result in key/val
hipError_t launch_finish_points(const double *xy, const double *w, int64_t n, const uint32_t *perm,
                                double cx, double cy, double s, int G, float *fr32, double *fr64,
                                double *wsorted, hipStream_t st);
// Debug validation of one binned point set (FEMNFFT_DEBUG_CHECKS): keys sorted and inside the
// cell table, cell starts consistent with the keys, fractions in [0, 1], perm a permutation of
// [0, n) (cnt: n scratch counters).  Adds the number of violations to *bad (zeroed here).
hipError_t launch_check_bins(const uint32_t *key, const uint32_t *perm, const uint32_t *cstart, const float *fr32,
                             const double *fr64, int64_t n, int64_t ncell, uint32_t *cnt, uint32_t *bad,
                             hipStream_t st);
// true when FEMNFFT_DEBUG_CHECKS is set to anything but "" or "0"
bool debug_checks_from_env();
hipError_t launch_cellstart(const uint32_t *key, int64_t n, int64_t ncell, uint32_t *cstart,
                            hipStream_t st);
// 2D binning: key holds cell * NEAR_SUB + x slice, sorted; writes the cell starts cstart
// [ncell + 1] and the slice starts csub [ncell NEAR_SUB + 1], then turns key into cell keys.
hipError_t launch_cellstart_sub(uint32_t *key, int64_t n, int64_t ncell, uint32_t *cstart, uint32_t *csub,
                                hipStream_t st);
// plan
hipError_t launch_kr_samples(double2 *a, int n, const double *coef, int p, double eps_I, double eps_B,
                             const double *cB, int ncB, hipStream_t st);
hipError_t launch_fft2d_c2c64(double2 *a, int n, const double2 *tw, hipStream_t st);
hipError_t launch_make_W(const double2 *bl, int n, const double *psihat, int precision, void *W,
                         hipStream_t st);
// charges / reductions
// val[c][k] = w_k q[perm_k][c] (ncomp 1 or 2); part (may be NULL): one sum of component 0
// per block launched, *nblk of them (at most 1024)
hipError_t launch_set_values(const double *q, const double *w, const uint32_t *perm, int64_t n,
                             int ncomp, int precision, void *val, double *val64, double *part, int *nblk,
                             hipStream_t st);
hipError_t launch_sum_partials(const double *part, int64_t np, double *red, hipStream_t st);
hipError_t launch_sum(const double *x, int64_t n, double *red, hipStream_t st);  // red[0] = sum
hipError_t launch_fill(double *x, int64_t n, double v, hipStream_t st);
// spread / fold / gather
hipError_t launch_spread(int precision, const Plan &P, const Geom &g, int set, const Buffers &b,
                         const void *val, int nfield, double *ptile, hipStream_t st);
hipError_t launch_fold(int precision, const Geom &g, int m, int tile, const double *ptile, int nfield, void *grid,
                       int64_t fstride, hipStream_t st);
hipError_t launch_gather(int precision, const Plan &P, const Geom &g, int set, const Buffers &b,
                         const void *grid, int nfield, int64_t fstride, double *far, int64_t farstride,
                         hipStream_t st);
// FFT passes
// Column pass over nclass multiplier tables (W0, and W1 when nclass = 2):
//   COL_FWD     inputs x_k, one per class: acc = sum_k W_k x_k; outputs acc and, with hy,
//               -2 pi i l_y acc
//   COL_ADJ_PHI input x: outputs W_k x, k < nclass
//   COL_ADJ_H   inputs x_0, x_1 (the two components): acc = sum_d 2 pi i l_d x_d;
//               outputs W_k acc, k < nclass
// The row pass writes the spectrum as spec[l_x][y] (ldS apart), or, with two fields,
// interleaved as spec[l_x][y][field]; the column pass reads it the same way (two inputs
// are always two interleaved fields) and writes its outputs ofstride apart.
enum ColMode { COL_FWD = 0, COL_ADJ_PHI = 1, COL_ADJ_H = 2 };
hipError_t launch_rows_fwd(int precision, int G, int nh, const void *grid, int64_t fstride, int Ex, int Ey,
                           int nfield, void *spec, int64_t ldS, const void *tw,
                           hipStream_t st);
hipError_t launch_cols(int precision, int G, int nh, const void *spec, void *out,
                       int64_t ofstride, int64_t ldS, int Ey, int mode, int nclass, int hy, const void *W0,
                       const void *W1, const void *tw, hipStream_t st);
// fwd: phi / H grids from T_phi (and T_Hy); adjoint: nout real grids from nout spectra
hipError_t launch_rows_inv(int precision, int G, int nh, const void *T, int64_t tfstride, int64_t ldS,
                           void *grid, int64_t fstride, int Ex, int Ey, int fwd, int want_phi, int want_h,
                           int nout, const void *tw, hipStream_t st);
// near field + final
struct NearArgs {
    double eps2g;        // eps_I^2 in grid units^2
    double inv_e2;       // 1 / eps2g
    double inv_eg;       // 1 / (eps_I G): the mixed path stages offsets in units of eps_I
    double ginv;         // 1/G
    // T_I(x) - K(eps_I) as a polynomial in x = (r/eps_I)^2: u_k = a_k, u_0 = a_0 - K(eps_I)
    double u[MAXP];
    double du[MAXP];     // U'(x) = T'(x): du_k = (k+1) u_{k+1}
    double lc[9];        // 1/(2k+1), k = 1..9 (series of the logarithm)
    double ln2hi, ln2lo; // ln 2 in two parts
    double czero;        // phi share of a coincident pair: -(a_0 + ln(s)/2pi)
    int p;
    int rnear;
    int f32;             // 1: the logarithm and reciprocal of x are evaluated in FP32 (mixed precision)
    double scale;        // s
    double offset;       // (ln s / 2 pi)
};
// forward: targets against source set in_set; accum = 0 writes far + near (+ the
// scale term of all charges), accum = 1 adds the near part only
hipError_t launch_near_fwd(const Geom &g, const Buffers &b, const NearArgs &na, const NearShape &sh, int in_set,
                           int accum, const double *sum_s, int want_phi, int want_h, double *phi, double *H,
                           const uint32_t *blocks, int nblocks, hipStream_t st);
// adjoint: source set out_set against the targets; u is that set's part of the output
hipError_t launch_near_adj(const Geom &g, const Buffers &b, const NearArgs &na, const NearShape &sh, int out_set,
                           int kind, const double *sum_v, double *u, const uint32_t *blocks, int nblocks,
                           hipStream_t st);
// The near field's home blocks (NBX x NBY cells) of the geometry, and the list of those with
// home points of out_set (and, if need_in, points of in_set within R cells): the sparse
// surface class runs only over these.  *count (device) receives the list length.
// near_blocks_bound(emax): the block count of any window of at most emax x emax cells
// for any allowed shape (the capacity of the lists).  Entries beyond cap are counted in
// *count but not written.
int near_blocks(const Geom &g, const NearShape &sh);
bool near_shape_ok(const NearShape &sh);
int64_t near_blocks_bound(int64_t emax);
hipError_t launch_block_list(const Geom &g, const Buffers &b, const NearShape &sh, int out_set, int in_set, int R,
                             int need_in, uint32_t *list, uint32_t cap, uint32_t *count, hipStream_t st);
hipError_t launch_near_coincident(const Geom &g, const Buffers &b, const NearArgs &na, int out_set, int in_set,
                                  double *out, hipStream_t st);
hipError_t launch_coincident_count(const Geom &g, const Buffers &b, int in_set, double *cnt, hipStream_t st);

// host helpers
double bessel_i0(double x);
void twiddles(int N, std::vector<double> &re, std::vector<double> &im);
// Pass-ordered twiddles of an N-point line (N a power of two, N >= 8), interleaved
// (re, im), max(N - 8, 1) entries: the layout fftd::fft_line_st reads.
void staged_twiddles(int N, std::vector<double> &t);

}  // namespace fn
