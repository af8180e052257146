// P1 finite-element front of the fast summation: quadrature sources, charge
// operator C and its transpose, lumped nodal mass, and the demagnetizing energy
// with its gradient (the paper's "Discretization" section: linear interpolation
// of M on triangles, volume density rho = -div M and surface density
// sigma = M.n, quadrature points with weights omega_j det J).
//
// Readings (the paper's quadrature footnote is missing): the volume rule has 3
// points at barycentric (2/3, 1/6, 1/6) and its permutations with weight |T|/3;
// the surface rule is 2-point Gauss-Legendre on each straight boundary edge with
// weight |e|/2; the outward normal of an edge (a, b) with the domain on its left
// is (dy, -dx)/|e|.  Source order: 3 volume points per triangle (triangle
// major), then 2 surface points per boundary edge.
//
// Energy: E = -1/2 sum_i l_i M_i . H_i with the lumped mass l_i = sum of |T|/3
// over the triangles at node i, and H = A C M (A: the H map of the fast sum).
// Its gradient is dE/dM = -1/2 (l H + C^T A^T (l M)).
//
// C^T and the lumped mass gather over a node -> (triangle corner | edge end)
// incidence list built once by a stable radix sort of the corner slots by node,
// so every sum runs in a fixed order (deterministic).  Everything is FP64.
#include "fn_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

namespace fn {
namespace {

constexpr double GL1 = 0.21132486540518711775;  // 1/2 - 1/(2 sqrt 3)
constexpr double GL2 = 0.78867513459481288225;  // 1/2 + 1/(2 sqrt 3)
constexpr double B_HI = 2.0 / 3.0, B_LO = 1.0 / 6.0;
constexpr int FB = 256;

// per-block sum of `bad` flags (grid-stride), partial per block
__device__ __forceinline__ void block_sum_store(double v, double *part)
{
    __shared__ double sh[FB];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = FB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Count out-of-range vertex indices and non-finite coordinates.
__global__ void __launch_bounds__(FB) k_validate(const double *__restrict__ nodes, int64_t N,
                                                 const int32_t *__restrict__ tris, int64_t T,
                                                 const int32_t *__restrict__ bedges, int64_t E,
                                                 double *__restrict__ part)
{
    double bad = 0.0;
    const int64_t stride = (int64_t)gridDim.x * FB;
    for (int64_t i = blockIdx.x * (int64_t)FB + threadIdx.x; i < 2 * N; i += stride)
        bad += isfinite(nodes[i]) ? 0.0 : 1.0;
    for (int64_t i = blockIdx.x * (int64_t)FB + threadIdx.x; i < 3 * T; i += stride)
        bad += (tris[i] >= 0 && tris[i] < N) ? 0.0 : 1.0;
    for (int64_t i = blockIdx.x * (int64_t)FB + threadIdx.x; i < 2 * E; i += stride)
        bad += (bedges[i] >= 0 && bedges[i] < N) ? 0.0 : 1.0;
    block_sum_store(bad, part);
}

// Triangle gradients of the hat functions and areas, SoA: tg[k T + t], k = 0..5
// for (g0x, g0y, g1x, g1y, g2x, g2y), k = 6 for |T|.  Counts degenerate triangles
// (twice the area at most 1e-12 of the magnitude of its two cross-product terms).
__global__ void __launch_bounds__(FB) k_tri_geom(const double *__restrict__ nodes, const int32_t *__restrict__ tris,
                                                 int64_t T, double *__restrict__ tg, double *__restrict__ part)
{
    double bad = 0.0;
    for (int64_t t = blockIdx.x * (int64_t)FB + threadIdx.x; t < T; t += (int64_t)gridDim.x * FB) {
        const int32_t i0 = tris[3 * t], i1 = tris[3 * t + 1], i2 = tris[3 * t + 2];
        const double x0 = nodes[2 * i0], y0 = nodes[2 * i0 + 1];
        const double x1 = nodes[2 * i1], y1 = nodes[2 * i1 + 1];
        const double x2 = nodes[2 * i2], y2 = nodes[2 * i2 + 1];
        const double p = (x1 - x0) * (y2 - y0), r = (y1 - y0) * (x2 - x0);
        const double a2 = p - r;
        // relative test: a repeated vertex leaves a rounding residual, not an exact zero
        bad += (fabs(a2) > 1e-12 * (fabs(p) + fabs(r)) && isfinite(a2)) ? 0.0 : 1.0;
        tg[0 * T + t] = (y1 - y2) / a2;
        tg[1 * T + t] = (x2 - x1) / a2;
        tg[2 * T + t] = (y2 - y0) / a2;
        tg[3 * T + t] = (x0 - x2) / a2;
        tg[4 * T + t] = (y0 - y1) / a2;
        tg[5 * T + t] = (x1 - x0) / a2;
        tg[6 * T + t] = 0.5 * fabs(a2);
    }
    block_sum_store(bad, part);
}

// Edge outward normals and lengths, SoA: eg[k E + e], k = 0, 1 normal, 2 length.
__global__ void __launch_bounds__(FB) k_edge_geom(const double *__restrict__ nodes, const int32_t *__restrict__ bedges,
                                                  int64_t E, double *__restrict__ eg, double *__restrict__ part)
{
    double bad = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)FB + threadIdx.x; e < E; e += (int64_t)gridDim.x * FB) {
        const int32_t ia = bedges[2 * e], ib = bedges[2 * e + 1];
        const double dx = nodes[2 * ib] - nodes[2 * ia], dy = nodes[2 * ib + 1] - nodes[2 * ia + 1];
        const double L = hypot(dx, dy);
        bad += (L > 0.0 && isfinite(L)) ? 0.0 : 1.0;
        eg[0 * E + e] = dy / L;
        eg[1 * E + e] = -dx / L;
        eg[2 * E + e] = L;
    }
    block_sum_store(bad, part);
}

// Quadrature points x [S][2] and weights w [S], S = 3T + 2E.
__global__ void k_sources(const double *__restrict__ nodes, const int32_t *__restrict__ tris, int64_t T,
                          const int32_t *__restrict__ bedges, int64_t E, const double *__restrict__ tg,
                          const double *__restrict__ eg, double *__restrict__ x, double *__restrict__ w)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= 3 * T + 2 * E) return;
    if (s < 3 * T) {
        const int64_t t = s / 3;
        const int k = (int)(s - 3 * t);
        const int32_t i0 = tris[3 * t], i1 = tris[3 * t + 1], i2 = tris[3 * t + 2];
        const double c0 = k == 0 ? B_HI : B_LO, c1 = k == 1 ? B_HI : B_LO, c2 = k == 2 ? B_HI : B_LO;
        x[2 * s] = (c0 * nodes[2 * i0] + c1 * nodes[2 * i1]) + c2 * nodes[2 * i2];
        x[2 * s + 1] = (c0 * nodes[2 * i0 + 1] + c1 * nodes[2 * i1 + 1]) + c2 * nodes[2 * i2 + 1];
        w[s] = tg[6 * T + t] / 3.0;
    } else {
        const int64_t r = s - 3 * T, e = r / 2;
        const double tq = (r & 1) ? GL2 : GL1;
        const int32_t ia = bedges[2 * e], ib = bedges[2 * e + 1];
        x[2 * s] = (1.0 - tq) * nodes[2 * ia] + tq * nodes[2 * ib];
        x[2 * s + 1] = (1.0 - tq) * nodes[2 * ia + 1] + tq * nodes[2 * ib + 1];
        w[s] = 0.5 * eg[2 * E + e];
    }
}

// Incidence keys: slot s < 3T is corner s % 3 of triangle s / 3 (node tris[s]);
// slot 3T + 2e + end is end `end` of boundary edge e (node bedges[2e + end]).
__global__ void k_inc_keys(const int32_t *__restrict__ tris, int64_t T, const int32_t *__restrict__ bedges, int64_t E,
                           uint32_t *__restrict__ key, uint32_t *__restrict__ slot)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= 3 * T + 2 * E) return;
    key[s] = (uint32_t)(s < 3 * T ? tris[s] : bedges[s - 3 * T]);
    slot[s] = (uint32_t)s;
}

__global__ void k_lumped(const uint32_t *__restrict__ off, const uint32_t *__restrict__ slot, int64_t N, int64_t T,
                         const double *__restrict__ tg, double *__restrict__ ell)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    double a = 0.0;
    for (uint32_t k = off[i]; k < off[i + 1]; ++k) {
        const uint32_t s = slot[k];
        if (s < 3 * T) a += tg[6 * T + s / 3] / 3.0;
    }
    ell[i] = a;
}

// q = C M: rho_T = -div M_h on the 3 volume points of T, sigma = M_h . n at the
// two Gauss points of each boundary edge.  One thread per triangle or edge.
__global__ void k_charges(const double *__restrict__ M, const int32_t *__restrict__ tris, int64_t T,
                          const int32_t *__restrict__ bedges, int64_t E, const double *__restrict__ tg,
                          const double *__restrict__ eg, double *__restrict__ q)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < T) {
        const int64_t t = k;
        const int32_t i0 = tris[3 * t], i1 = tris[3 * t + 1], i2 = tris[3 * t + 2];
        const double d0 = M[2 * i0] * tg[0 * T + t] + M[2 * i0 + 1] * tg[1 * T + t];
        const double d1 = M[2 * i1] * tg[2 * T + t] + M[2 * i1 + 1] * tg[3 * T + t];
        const double d2 = M[2 * i2] * tg[4 * T + t] + M[2 * i2 + 1] * tg[5 * T + t];
        const double rho = -((d0 + d1) + d2);
        q[3 * t] = rho;
        q[3 * t + 1] = rho;
        q[3 * t + 2] = rho;
    } else if (k < T + E) {
        const int64_t e = k - T;
        const int32_t ia = bedges[2 * e], ib = bedges[2 * e + 1];
        const double nx = eg[0 * E + e], ny = eg[1 * E + e];
        for (int c = 0; c < 2; ++c) {
            const double tq = c ? GL2 : GL1;
            const double mx = (1.0 - tq) * M[2 * ia] + tq * M[2 * ib];
            const double my = (1.0 - tq) * M[2 * ia + 1] + tq * M[2 * ib + 1];
            q[3 * T + 2 * e + c] = mx * nx + my * ny;
        }
    }
}

// out_i = (C^T u)_i, or with GRAD: out_i = -1/2 (l_i H_i + (C^T u)_i).
template <bool GRAD>
__global__ void k_charges_T(const uint32_t *__restrict__ off, const uint32_t *__restrict__ slot, int64_t N, int64_t T,
                            int64_t E, const double *__restrict__ tg, const double *__restrict__ eg,
                            const double *__restrict__ u, const double *__restrict__ ell,
                            const double *__restrict__ H, double *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    double ox = 0.0, oy = 0.0;
    for (uint32_t k = off[i]; k < off[i + 1]; ++k) {
        const int64_t s = slot[k];
        if (s < 3 * T) {
            const int64_t t = s / 3;
            const int c = (int)(s - 3 * t);
            const double us = (u[3 * t] + u[3 * t + 1]) + u[3 * t + 2];
            ox -= us * tg[(2 * c) * T + t];
            oy -= us * tg[(2 * c + 1) * T + t];
        } else {
            const int64_t r = s - 3 * T, e = r / 2;
            const bool end1 = r & 1;
            const double u0 = u[3 * T + 2 * e], u1 = u[3 * T + 2 * e + 1];
            const double a = end1 ? GL1 * u0 + GL2 * u1 : (1.0 - GL1) * u0 + (1.0 - GL2) * u1;
            ox += a * eg[0 * E + e];
            oy += a * eg[1 * E + e];
        }
    }
    if (GRAD) {
        out[2 * i] = -0.5 * (ell[i] * H[2 * i] + ox);
        out[2 * i + 1] = -0.5 * (ell[i] * H[2 * i + 1] + oy);
    } else {
        out[2 * i] = ox;
        out[2 * i + 1] = oy;
    }
}

// e_i = l_i M_i . H_i and V_i = l_i M_i.
__global__ void k_energy_terms(const double *__restrict__ M, const double *__restrict__ H,
                               const double *__restrict__ ell, int64_t N, double *__restrict__ e,
                               double *__restrict__ V)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double mx = M[2 * i], my = M[2 * i + 1];
    e[i] = ell[i] * (mx * H[2 * i] + my * H[2 * i + 1]);
    if (V) {
        V[2 * i] = ell[i] * mx;
        V[2 * i + 1] = ell[i] * my;
    }
}

// V_i = l_i M_i alone (the adjoint's input needs M, not H)
__global__ void k_lumped_V(const double *__restrict__ M, const double *__restrict__ ell, int64_t N,
                           double *__restrict__ V)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    V[2 * i] = ell[i] * M[2 * i];
    V[2 * i + 1] = ell[i] * M[2 * i + 1];
}

__global__ void k_half_neg(const double *__restrict__ sum, double *__restrict__ E)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) E[0] = -0.5 * sum[0];
}

__global__ void k_half(const double *__restrict__ sum, double *__restrict__ E)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) E[0] = 0.5 * sum[0];
}

// Charge form at the quadrature points: e_j = w_j q_j phi_j (summed for E_q = 1/2 sum e_j)
// and u_j = w_j phi_j (dE_q/dq_j: the potential matrix between distinct points is
// symmetric, so the gradient with respect to M is C^T u).
__global__ void k_charge_energy_terms(const double *__restrict__ w, const double *__restrict__ q,
                                      const double *__restrict__ phi, int64_t S, double *__restrict__ e,
                                      double *__restrict__ u)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= S) return;
    const double wp = w[j] * phi[j];
    u[j] = wp;
    e[j] = q[j] * wp;
}

// -grad of the P1 interpolant of nodal phi on triangle t: -(phi_0 g_0 + phi_1 g_1 + phi_2 g_2)
__device__ __forceinline__ double2 p1_grad(const double *__restrict__ phi, const int32_t *__restrict__ tris,
                                           const double *__restrict__ tg, int64_t T, int64_t t)
{
    const double f0 = phi[tris[3 * t]], f1 = phi[tris[3 * t + 1]], f2 = phi[tris[3 * t + 2]];
    const double gx = (f0 * tg[0 * T + t] + f1 * tg[2 * T + t]) + f2 * tg[4 * T + t];
    const double gy = (f0 * tg[1 * T + t] + f1 * tg[3 * T + t]) + f2 * tg[5 * T + t];
    return make_double2(-gx, -gy);
}

__global__ void k_p1_grad_tri(const double *__restrict__ phi, const int32_t *__restrict__ tris,
                              const double *__restrict__ tg, int64_t T, double *__restrict__ H)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= T) return;
    const double2 h = p1_grad(phi, tris, tg, T, t);
    H[2 * t] = h.x;
    H[2 * t + 1] = h.y;
}

// Lumped projection onto the nodes: H_i = (1/l_i) sum over the triangles at i of (|T|/3) H_T,
// in the fixed order of the node's incidence list (edge slots carry no area).
__global__ void k_p1_grad_node(const uint32_t *__restrict__ off, const uint32_t *__restrict__ slot, int64_t N,
                               int64_t T, const double *__restrict__ phi, const int32_t *__restrict__ tris,
                               const double *__restrict__ tg, const double *__restrict__ ell, double *__restrict__ H)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    double hx = 0.0, hy = 0.0;
    for (uint32_t k = off[i]; k < off[i + 1]; ++k) {
        const uint32_t s = slot[k];
        if (s >= 3 * T) continue;
        const int64_t t = s / 3;
        const double a3 = tg[6 * T + t] / 3.0;
        const double2 h = p1_grad(phi, tris, tg, T, t);
        hx += a3 * h.x;
        hy += a3 * h.y;
    }
    const double l = ell[i];
    H[2 * i] = l > 0.0 ? hx / l : 0.0;
    H[2 * i + 1] = l > 0.0 ? hy / l : 0.0;
}

inline int nb_of(int64_t n) { return (int)((n + FB - 1) / FB); }
inline int nb_grid(int64_t n) { return (int)std::min<int64_t>(256, std::max<int64_t>(1, (n + FB - 1) / FB)); }

}  // namespace
}  // namespace fn

using namespace fn;

// ---------------------------------------------------------------------------
// mesh object

struct MeshBuf {
    double *nodes = nullptr, *tg = nullptr, *eg = nullptr, *ell = nullptr, *x = nullptr, *w = nullptr;
    double *q = nullptr, *H = nullptr, *V = nullptr, *u = nullptr, *e = nullptr, *red = nullptr;
    double *es = nullptr, *phis = nullptr;  // charge form: terms w q phi, potential at the sources
    int32_t *tris = nullptr, *bedges = nullptr;
    uint32_t *off = nullptr, *slot = nullptr, *key = nullptr, *skey = nullptr, *sval = nullptr, *hist = nullptr;
};

struct fn_mesh {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t N = 0, T = 0, E = 0, S = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    MeshBuf b;
    bool ready = false;
    uint64_t stamp = 0;
    std::string err;
};

static constexpr int MESH_RED = 2048;  // doubles of reduction scratch

static size_t mesh_layout(const fn_mesh *m, MeshBuf *b, char *base)
{
    const int64_t N = std::max<int64_t>(m->N, 1), T = std::max<int64_t>(m->T, 1), E = std::max<int64_t>(m->E, 1);
    const int64_t S = 3 * T + 2 * E;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = (o + bytes + 255) & ~(size_t)255;
        return base ? base + r : nullptr;
    };
    MeshBuf t;
    t.nodes = (double *)take(16 * N);
    t.tris = (int32_t *)take(12 * T);
    t.bedges = (int32_t *)take(8 * E);
    t.tg = (double *)take(56 * T);
    t.eg = (double *)take(24 * E);
    t.ell = (double *)take(8 * N);
    t.off = (uint32_t *)take(4 * (N + 1));
    t.slot = (uint32_t *)take(4 * S);
    t.key = (uint32_t *)take(4 * S);
    t.skey = (uint32_t *)take(4 * S);
    t.sval = (uint32_t *)take(4 * S);
    t.hist = (uint32_t *)take(4 * 256 * ((S + 4095) / 4096));
    t.x = (double *)take(16 * S);
    t.w = (double *)take(8 * S);
    t.q = (double *)take(8 * S);
    t.u = (double *)take(8 * S);
    t.H = (double *)take(16 * N);
    t.V = (double *)take(16 * N);
    t.e = (double *)take(8 * N);
    t.es = (double *)take(8 * S);
    t.phis = (double *)take(8 * S);
    t.red = (double *)take(8 * MESH_RED);
    if (b) *b = t;
    return o;
}

#define MESH_ERR(mh, code, msg)  \
    do {                         \
        (mh)->err = (msg);       \
        return (code);           \
    } while (0)

#define MESH_HIP(mh, call)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            (mh)->err = std::string("HIP error in ") + #call + ": " + hipGetErrorString(e_);     \
            return FN_E_DEVICE;                                                                  \
        }                                                                                        \
    } while (0)

static thread_local std::string g_mesh_create_err;

static int mesh_select_device(fn_mesh *m)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) MESH_ERR(m, FN_E_DEVICE, std::string("pending HIP error: ") + hipGetErrorString(e));
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != m->device)
        if (hipSetDevice(m->device) != hipSuccess) MESH_ERR(m, FN_E_DEVICE, "cannot select the mesh's device");
    return FN_OK;
}

// sum of the first nblk block partials at part (host read-back; set-up only)
static int read_bad(fn_mesh *m, const double *part, int nblk, double *out)
{
    std::vector<double> h(nblk);
    MESH_HIP(m, hipMemcpyAsync(h.data(), part, sizeof(double) * nblk, hipMemcpyDeviceToHost, m->stream));
    MESH_HIP(m, hipStreamSynchronize(m->stream));
    double s = 0.0;
    for (double v : h) s += v;
    *out = s;
    return FN_OK;
}

extern "C" {

int fn_mesh_create(int64_t n_nodes, int64_t n_tris, int64_t n_bedges, void *stream, fn_mesh **out)
{
    if (!out) { g_mesh_create_err = "out is NULL"; return FN_E_INVAL; }
    *out = nullptr;
    if (n_nodes < 3 || n_tris < 1 || n_bedges < 0 || n_nodes >= ((int64_t)1 << 31) ||
        3 * n_tris + 2 * n_bedges >= ((int64_t)1 << 31)) {
        g_mesh_create_err = "need n_nodes >= 3, n_tris >= 1, n_bedges >= 0, nodes and 3 n_tris + 2 n_bedges < 2^31";
        return FN_E_INVAL;
    }
    fn_mesh *m = new (std::nothrow) fn_mesh();
    if (!m) { g_mesh_create_err = "out of host memory"; return FN_E_NOMEM; }
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        g_mesh_create_err = "no HIP device";
        return FN_E_DEVICE;
    }
    m->stream = static_cast<hipStream_t>(stream);
    m->N = n_nodes;
    m->T = n_tris;
    m->E = n_bedges;
    m->S = 3 * n_tris + 2 * n_bedges;
    *out = m;
    return FN_OK;
}

int fn_mesh_destroy(fn_mesh *mesh)
{
    delete mesh;
    return FN_OK;
}

int fn_mesh_workspace_size(const fn_mesh *mesh, size_t *bytes)
{
    if (!mesh || !bytes) return FN_E_INVAL;
    *bytes = mesh_layout(mesh, nullptr, nullptr);
    return FN_OK;
}

int fn_mesh_set_workspace(fn_mesh *mesh, void *dev_ptr, size_t bytes)
{
    if (!mesh) return FN_E_INVAL;
    if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255))
        MESH_ERR(mesh, FN_E_INVAL, "workspace must be non-NULL and 256-byte aligned");
    const size_t need = mesh_layout(mesh, nullptr, nullptr);
    if (bytes < need) MESH_ERR(mesh, FN_E_NOMEM, "mesh workspace too small");
    mesh->ws = dev_ptr;
    mesh->ws_bytes = bytes;
    mesh_layout(mesh, &mesh->b, static_cast<char *>(dev_ptr));
    mesh->ready = false;
    return FN_OK;
}

int fn_mesh_set(fn_mesh *mesh, const double *nodes, const int32_t *tris, const int32_t *bedges)
{
    if (!mesh) return FN_E_INVAL;
    fn_mesh *m = mesh;
    if (!m->ws) MESH_ERR(m, FN_E_STATE, "fn_mesh_set_workspace must be called before fn_mesh_set");
    if (!nodes || !tris || (m->E > 0 && !bedges)) MESH_ERR(m, FN_E_INVAL, "NULL mesh array");
    if (stream_capturing(m->stream)) MESH_ERR(m, FN_E_STATE, "fn_mesh_set waits for the device: not allowed during graph capture");
    int rc = mesh_select_device(m);
    if (rc) return rc;
    m->ready = false;
    const MeshBuf &b = m->b;
    hipStream_t st = m->stream;
    MESH_HIP(m, hipMemcpyAsync(b.nodes, nodes, 16 * m->N, hipMemcpyDeviceToDevice, st));
    MESH_HIP(m, hipMemcpyAsync(b.tris, tris, 12 * m->T, hipMemcpyDeviceToDevice, st));
    if (m->E > 0) MESH_HIP(m, hipMemcpyAsync(b.bedges, bedges, 8 * m->E, hipMemcpyDeviceToDevice, st));
    const int nv = nb_grid(std::max<int64_t>(2 * m->N, std::max<int64_t>(3 * m->T, 2 * m->E)));
    k_validate<<<nv, FB, 0, st>>>(b.nodes, m->N, b.tris, m->T, b.bedges, m->E, b.red);
    MESH_HIP(m, hipGetLastError());
    double bad = 0.0;
    rc = read_bad(m, b.red, nv, &bad);
    if (rc) return rc;
    if (bad > 0.0) MESH_ERR(m, FN_E_INVAL, "vertex index out of range or non-finite node coordinate");
    const int nt = nb_grid(m->T), ne = nb_grid(m->E);
    k_tri_geom<<<nt, FB, 0, st>>>(b.nodes, b.tris, m->T, b.tg, b.red);
    k_edge_geom<<<ne, FB, 0, st>>>(b.nodes, b.bedges, m->E, b.eg, b.red + 256);
    MESH_HIP(m, hipGetLastError());
    double bad_t = 0.0, bad_e = 0.0;
    rc = read_bad(m, b.red, nt, &bad_t);
    if (rc) return rc;
    if (m->E > 0) {
        rc = read_bad(m, b.red + 256, ne, &bad_e);
        if (rc) return rc;
    }
    if (bad_t > 0.0) MESH_ERR(m, FN_E_DOMAIN, "degenerate triangle (zero area)");
    if (bad_e > 0.0) MESH_ERR(m, FN_E_DOMAIN, "degenerate boundary edge (zero length)");
    // incidence list: slots sorted by node (stable, so by slot within a node)
    k_inc_keys<<<nb_of(m->S), FB, 0, st>>>(b.tris, m->T, b.bedges, m->E, b.key, b.slot);
    MESH_HIP(m, hipGetLastError());
    int keybits = 1;
    while (((int64_t)1 << keybits) < m->N) ++keybits;
    MESH_HIP(m, radix_sort(b.key, b.slot, b.skey, b.sval, b.hist, m->S, keybits, st));
    MESH_HIP(m, launch_cellstart(b.key, m->S, m->N, b.off, st));
    k_lumped<<<nb_of(m->N), FB, 0, st>>>(b.off, b.slot, m->N, m->T, b.tg, b.ell);
    k_sources<<<nb_of(m->S), FB, 0, st>>>(b.nodes, b.tris, m->T, b.bedges, m->E, b.tg, b.eg, b.x, b.w);
    MESH_HIP(m, hipGetLastError());
    MESH_HIP(m, hipStreamSynchronize(st));
    m->ready = true;
    m->stamp++;
    return FN_OK;
}

static int mesh_ready(fn_mesh *m)
{
    if (!m->ready) MESH_ERR(m, FN_E_STATE, "fn_mesh_set must succeed first");
    return mesh_select_device(m);
}

int fn_mesh_sources(fn_mesh *mesh, double *x, double *w)
{
    if (!mesh) return FN_E_INVAL;
    int rc = mesh_ready(mesh);
    if (rc) return rc;
    if (!x && !w) MESH_ERR(mesh, FN_E_INVAL, "both outputs are NULL");
    if (x) MESH_HIP(mesh, hipMemcpyAsync(x, mesh->b.x, 16 * mesh->S, hipMemcpyDeviceToDevice, mesh->stream));
    if (w) MESH_HIP(mesh, hipMemcpyAsync(w, mesh->b.w, 8 * mesh->S, hipMemcpyDeviceToDevice, mesh->stream));
    return FN_OK;
}

int fn_mesh_lumped_mass(fn_mesh *mesh, double *ell)
{
    if (!mesh) return FN_E_INVAL;
    int rc = mesh_ready(mesh);
    if (rc) return rc;
    if (!ell) MESH_ERR(mesh, FN_E_INVAL, "ell is NULL");
    MESH_HIP(mesh, hipMemcpyAsync(ell, mesh->b.ell, 8 * mesh->N, hipMemcpyDeviceToDevice, mesh->stream));
    return FN_OK;
}

static hipError_t launch_charges(const fn_mesh *m, const double *M, double *q, hipStream_t st)
{
    k_charges<<<nb_of(m->T + m->E), FB, 0, st>>>(M, m->b.tris, m->T, m->b.bedges, m->E, m->b.tg, m->b.eg, q);
    return hipGetLastError();
}

int fn_mesh_charges(fn_mesh *mesh, const double *M, double *q)
{
    if (!mesh) return FN_E_INVAL;
    int rc = mesh_ready(mesh);
    if (rc) return rc;
    if (!M || !q) MESH_ERR(mesh, FN_E_INVAL, "NULL M or q");
    MESH_HIP(mesh, launch_charges(mesh, M, q, mesh->stream));
    return FN_OK;
}

int fn_mesh_charges_T(fn_mesh *mesh, const double *u, double *out)
{
    if (!mesh) return FN_E_INVAL;
    int rc = mesh_ready(mesh);
    if (rc) return rc;
    if (!u || !out) MESH_ERR(mesh, FN_E_INVAL, "NULL u or out");
    const MeshBuf &b = mesh->b;
    k_charges_T<false><<<nb_of(mesh->N), FB, 0, mesh->stream>>>(b.off, b.slot, mesh->N, mesh->T, mesh->E, b.tg, b.eg,
                                                               u, nullptr, nullptr, out);
    MESH_HIP(mesh, hipGetLastError());
    return FN_OK;
}

int fn_bind_mesh(fn_ctx *ctx, fn_mesh *mesh)
{
    if (!ctx || !mesh) return FN_E_INVAL;
    if (!mesh->ready) {
        ctx->err = "fn_mesh_set must succeed before fn_bind_mesh";
        return FN_E_STATE;
    }
    if (mesh->device != ctx->device) {
        ctx->err = "mesh and context live on different devices";
        return FN_E_INVAL;
    }
    ctx->mesh = nullptr;
    // sources: 3 volume points per triangle, then 2 surface points per boundary edge
    int rc = fn_set_geometry_split(ctx, mesh->N, mesh->b.nodes, mesh->S, mesh->b.x, mesh->b.w, 2 * mesh->E);
    if (rc) return rc;
    ctx->mesh = mesh;
    ctx->mesh_stamp = mesh->stamp;
    ctx->mesh_at_sources = false;
    return FN_OK;
}

int fn_bind_mesh_sources(fn_ctx *ctx, fn_mesh *mesh)
{
    if (!ctx || !mesh) return FN_E_INVAL;
    if (!mesh->ready) {
        ctx->err = "fn_mesh_set must succeed before fn_bind_mesh_sources";
        return FN_E_STATE;
    }
    if (mesh->device != ctx->device) {
        ctx->err = "mesh and context live on different devices";
        return FN_E_INVAL;
    }
    ctx->mesh = nullptr;
    // targets = sources = the quadrature points, one source class: every source takes the
    // kernel regularized at eps_I, so the fast potential matrix is symmetric like the exact
    // one (with the boundary points as a class of their own, A[i][j] = K_{class of j} would
    // not be) and C^T (w phi) is the exact gradient of the energy evaluated; the potential
    // (unlike the field) of line charges converges at the volume radius too
    int rc = fn_set_geometry(ctx, mesh->S, mesh->b.x, mesh->S, mesh->b.x, mesh->b.w);
    if (rc) return rc;
    ctx->mesh = mesh;
    ctx->mesh_stamp = mesh->stamp;
    ctx->mesh_at_sources = true;
    return FN_OK;
}

int fn_energy_charge(fn_ctx *ctx, fn_mesh *mesh, const double *M, double *E, double *grad, double *phi_s)
{
    if (!ctx || !mesh) return FN_E_INVAL;
    if (!M || !E) {
        ctx->err = "NULL M or E";
        return FN_E_INVAL;
    }
    if (ctx->mesh != mesh || !ctx->mesh_at_sources || ctx->mesh_stamp != mesh->stamp || !mesh->ready ||
        !ctx->geom_ready) {
        ctx->err = "fn_bind_mesh_sources(ctx, mesh) must succeed after the last fn_mesh_set and fn_set_geometry";
        return FN_E_STATE;
    }
    hipStream_t st = ctx->stream;
    const MeshBuf &b = mesh->b;
    int rc = ctx_hip(ctx, launch_charges(mesh, M, b.q, st));
    if (rc) return rc;
    rc = fn_set_charges(ctx, b.q);
    if (rc) return rc;
    double *phi = phi_s ? phi_s : b.phis;
    rc = fn_eval_phi(ctx, phi);
    if (rc) return rc;
    k_charge_energy_terms<<<nb_of(mesh->S), FB, 0, st>>>(b.w, b.q, phi, mesh->S, b.es, b.u);
    rc = ctx_hip(ctx, hipGetLastError());
    if (rc) return rc;
    rc = ctx_hip(ctx, launch_sum(b.es, mesh->S, b.red, st));
    if (rc) return rc;
    k_half<<<1, 64, 0, st>>>(b.red, E);
    rc = ctx_hip(ctx, hipGetLastError());
    if (rc || !grad) return rc;
    k_charges_T<false><<<nb_of(mesh->N), FB, 0, st>>>(b.off, b.slot, mesh->N, mesh->T, mesh->E, b.tg, b.eg, b.u,
                                                      nullptr, nullptr, grad);
    return ctx_hip(ctx, hipGetLastError());
}

int fn_mesh_p1_gradient(fn_mesh *mesh, const double *phi, double *H_tri, double *H_node)
{
    if (!mesh) return FN_E_INVAL;
    int rc = mesh_ready(mesh);
    if (rc) return rc;
    if (!phi || (!H_tri && !H_node)) MESH_ERR(mesh, FN_E_INVAL, "NULL phi, or both outputs NULL");
    const MeshBuf &b = mesh->b;
    if (H_tri) k_p1_grad_tri<<<nb_of(mesh->T), FB, 0, mesh->stream>>>(phi, b.tris, b.tg, mesh->T, H_tri);
    if (H_node)
        k_p1_grad_node<<<nb_of(mesh->N), FB, 0, mesh->stream>>>(b.off, b.slot, mesh->N, mesh->T, phi, b.tris, b.tg,
                                                                b.ell, H_node);
    MESH_HIP(mesh, hipGetLastError());
    return FN_OK;
}

int fn_energy(fn_ctx *ctx, fn_mesh *mesh, const double *M, double *E, double *grad)
{
    if (!ctx || !mesh) return FN_E_INVAL;
    if (!M || !E) {
        ctx->err = "NULL M or E";
        return FN_E_INVAL;
    }
    if (ctx->mesh != mesh || ctx->mesh_at_sources || ctx->mesh_stamp != mesh->stamp || !mesh->ready ||
        !ctx->geom_ready) {
        ctx->err = "fn_bind_mesh(ctx, mesh) must succeed after the last fn_mesh_set and fn_set_geometry";
        return FN_E_STATE;
    }
    hipStream_t st = ctx->stream;
    const MeshBuf &b = mesh->b;
    int rc = ctx_hip(ctx, launch_charges(mesh, M, b.q, st));
    if (rc) return rc;
    rc = fn_set_charges(ctx, b.q);
    if (rc) return rc;
    // with the gradient, H and the H adjoint of V = l M run at once (fn_eval_with_H_adjoint),
    // unless that call would have to create its stream under graph capture
    const bool fused = grad && (ctx->stream2 || !stream_capturing(st));
    if (fused) {
        k_lumped_V<<<nb_of(mesh->N), FB, 0, st>>>(M, b.ell, mesh->N, b.V);
        rc = ctx_hip(ctx, hipGetLastError());
        if (rc) return rc;
        rc = fn_eval_with_H_adjoint(ctx, nullptr, b.H, b.V, b.u);
    } else {
        rc = fn_eval_H(ctx, b.H);
    }
    if (rc) return rc;
    k_energy_terms<<<nb_of(mesh->N), FB, 0, st>>>(M, b.H, b.ell, mesh->N, b.e, fused ? nullptr : b.V);
    rc = ctx_hip(ctx, hipGetLastError());
    if (rc) return rc;
    rc = ctx_hip(ctx, launch_sum(b.e, mesh->N, b.red, st));
    if (rc) return rc;
    k_half_neg<<<1, 64, 0, st>>>(b.red, E);
    rc = ctx_hip(ctx, hipGetLastError());
    if (rc) return rc;
    if (!grad) return FN_OK;
    if (!fused) {
        rc = fn_eval_H_adjoint(ctx, b.V, b.u);
        if (rc) return rc;
    }
    k_charges_T<true><<<nb_of(mesh->N), FB, 0, st>>>(b.off, b.slot, mesh->N, mesh->T, mesh->E, b.tg, b.eg, b.u, b.ell,
                                                     b.H, grad);
    return ctx_hip(ctx, hipGetLastError());
}

const char *fn_mesh_last_error(const fn_mesh *mesh)
{
    if (!mesh) return g_mesh_create_err.c_str();
    return mesh->err.c_str();
}

}  // extern "C"
