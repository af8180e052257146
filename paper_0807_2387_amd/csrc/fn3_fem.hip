// P1 finite-element front of the 3D fast summation on tetrahedra: quadrature sources,
// the charge operator C and its transpose, lumped nodal mass, and the demagnetizing
// energy with its gradient -- the 2D front of fn_fem.hip with tetrahedra and boundary
// triangles (the paper's "Discretization" section: linear interpolation of M in each
// element, rho = -div M inside, sigma = M.n on the boundary, quadrature points with
// weights omega_j det J).
//
// Readings (the paper's quadrature footnote is missing; its formulation holds in 3D
// alike): the volume rule has 4 points at barycentric (a, b, b, b) and permutations,
// a = (5 + 3 sqrt 5)/20, b = (5 - sqrt 5)/20, weight |T|/4 each (degree 2); the surface
// rule has 3 points at barycentric (2/3, 1/6, 1/6) and permutations, weight |F|/3 each;
// a boundary triangle (a, b, c) has the outward normal (b - a) x (c - a)/|.|.  Source
// order: 4 volume points per tetrahedron (tetrahedron major), then 3 surface points per
// boundary triangle.  Energy: E = -1/2 sum_i l_i M_i . H_i, l_i = sum of |T|/4 over the
// tetrahedra at node i, gradient -1/2 (l H + C^T A^T (l M)).
//
// C^T and the lumped mass gather over a node -> (tetrahedron corner | face corner)
// incidence list built by a stable radix sort of the corner slots by node, so every sum
// runs in a fixed order (deterministic).  Everything is FP64.
#include "fn_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace fn3m {

constexpr double QA = 0.58541019662496845446;   // (5 + 3 sqrt 5)/20
constexpr double QB = 0.13819660112501051518;   // (5 - sqrt 5)/20
constexpr double FHI = 2.0 / 3.0, FLO = 1.0 / 6.0;
constexpr int FB = 256;
constexpr int MESH_RED = 2048;

inline int nb_of(int64_t n) { return (int)std::max<int64_t>(1, (n + FB - 1) / FB); }
inline int nb_grid(int64_t n) { return (int)std::min<int64_t>(256, std::max<int64_t>(1, (n + FB - 1) / FB)); }

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

// out-of-range vertex indices and non-finite coordinates
__global__ void __launch_bounds__(FB) k3m_validate(const double *__restrict__ nodes, int64_t N,
                                                   const int32_t *__restrict__ tets, int64_t T,
                                                   const int32_t *__restrict__ faces, int64_t F, double *__restrict__ part)
{
    double bad = 0.0;
    const int64_t stride = (int64_t)gridDim.x * FB;
    for (int64_t i = blockIdx.x * (int64_t)FB + threadIdx.x; i < 3 * N; i += stride) bad += isfinite(nodes[i]) ? 0.0 : 1.0;
    for (int64_t i = blockIdx.x * (int64_t)FB + threadIdx.x; i < 4 * T; i += stride)
        bad += (tets[i] >= 0 && tets[i] < N) ? 0.0 : 1.0;
    for (int64_t i = blockIdx.x * (int64_t)FB + threadIdx.x; i < 3 * F; i += stride)
        bad += (faces[i] >= 0 && faces[i] < N) ? 0.0 : 1.0;
    block_sum_store(bad, part);
}

__device__ __forceinline__ void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// Gradients of the barycentric functions and volumes, SoA: tg[k T + t], k = 3 c + d for
// corner c's gradient component d (k < 12), k = 12 for |T|.  With the edge matrix
// J = [e1 e2 e3], e_k = p_k - p_0, the rows of J^{-1} are (e2 x e3, e3 x e1, e1 x e2)/det J,
// the gradients of lambda_1..3; lambda_0's is minus their sum.  Counts degenerate
// tetrahedra (|det J| at most 1e-12 of |e1||e2||e3|).
__global__ void __launch_bounds__(FB) k3m_tet_geom(const double *__restrict__ nodes, const int32_t *__restrict__ tets,
                                                   int64_t T, double *__restrict__ tg, double *__restrict__ part)
{
    double bad = 0.0;
    for (int64_t t = blockIdx.x * (int64_t)FB + threadIdx.x; t < T; t += (int64_t)gridDim.x * FB) {
        double p[4][3];
        for (int c = 0; c < 4; ++c)
            for (int d = 0; d < 3; ++d) p[c][d] = nodes[3 * (int64_t)tets[4 * t + c] + d];
        double e[3][3];
        for (int k = 0; k < 3; ++k)
            for (int d = 0; d < 3; ++d) e[k][d] = p[k + 1][d] - p[0][d];
        double r[3][3];
        cross3(e[1], e[2], r[0]);
        cross3(e[2], e[0], r[1]);
        cross3(e[0], e[1], r[2]);
        const double det = (e[0][0] * r[0][0] + e[0][1] * r[0][1]) + e[0][2] * r[0][2];
        const double scale = sqrt((e[0][0] * e[0][0] + e[0][1] * e[0][1] + e[0][2] * e[0][2]) *
                                  (e[1][0] * e[1][0] + e[1][1] * e[1][1] + e[1][2] * e[1][2]) *
                                  (e[2][0] * e[2][0] + e[2][1] * e[2][1] + e[2][2] * e[2][2]));
        bad += (fabs(det) > 1e-12 * scale && isfinite(det)) ? 0.0 : 1.0;
        for (int d = 0; d < 3; ++d) {
            const double g1 = r[0][d] / det, g2 = r[1][d] / det, g3 = r[2][d] / det;
            tg[(0 + d) * T + t] = -((g1 + g2) + g3);
            tg[(3 + d) * T + t] = g1;
            tg[(6 + d) * T + t] = g2;
            tg[(9 + d) * T + t] = g3;
        }
        tg[12 * T + t] = fabs(det) / 6.0;
    }
    block_sum_store(bad, part);
}

// Face unit normals and areas, SoA: fg[k F + f], k < 3 normal, k = 3 area.
__global__ void __launch_bounds__(FB) k3m_face_geom(const double *__restrict__ nodes, const int32_t *__restrict__ faces,
                                                    int64_t F, double *__restrict__ fg, double *__restrict__ part)
{
    double bad = 0.0;
    for (int64_t f = blockIdx.x * (int64_t)FB + threadIdx.x; f < F; f += (int64_t)gridDim.x * FB) {
        double a[3], b[3], c[3];
        for (int d = 0; d < 3; ++d) {
            const double a0 = nodes[3 * (int64_t)faces[3 * f] + d];
            a[d] = a0;
            b[d] = nodes[3 * (int64_t)faces[3 * f + 1] + d] - a0;
            c[d] = nodes[3 * (int64_t)faces[3 * f + 2] + d] - a0;
        }
        double n[3];
        cross3(b, c, n);
        const double a2 = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        bad += (a2 > 0.0 && isfinite(a2)) ? 0.0 : 1.0;
        for (int d = 0; d < 3; ++d) fg[d * F + f] = n[d] / a2;
        fg[3 * F + f] = 0.5 * a2;
    }
    block_sum_store(bad, part);
}

// Quadrature points x [S][3] and weights w [S], S = 4T + 3F.
__global__ void k3m_sources(const double *__restrict__ nodes, const int32_t *__restrict__ tets, int64_t T,
                            const int32_t *__restrict__ faces, int64_t F, const double *__restrict__ tg,
                            const double *__restrict__ fg, double *__restrict__ x, double *__restrict__ w)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= 4 * T + 3 * F) return;
    if (s < 4 * T) {
        const int64_t t = s / 4;
        const int k = (int)(s - 4 * t);
        for (int d = 0; d < 3; ++d) {
            double acc = 0.0;
            for (int c = 0; c < 4; ++c) acc += (c == k ? QA : QB) * nodes[3 * (int64_t)tets[4 * t + c] + d];
            x[3 * s + d] = acc;
        }
        w[s] = tg[12 * T + t] / 4.0;
    } else {
        const int64_t r = s - 4 * T, f = r / 3;
        const int k = (int)(r - 3 * f);
        for (int d = 0; d < 3; ++d) {
            double acc = 0.0;
            for (int c = 0; c < 3; ++c) acc += (c == k ? FHI : FLO) * nodes[3 * (int64_t)faces[3 * f + c] + d];
            x[3 * s + d] = acc;
        }
        w[s] = fg[3 * F + f] / 3.0;
    }
}

// incidence keys: slot s < 4T is corner s % 4 of tetrahedron s / 4; slot 4T + 3f + k is
// corner k of boundary face f
__global__ void k3m_inc_keys(const int32_t *__restrict__ tets, int64_t T, const int32_t *__restrict__ faces, int64_t F,
                             uint32_t *__restrict__ key, uint32_t *__restrict__ slot)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= 4 * T + 3 * F) return;
    key[s] = (uint32_t)(s < 4 * T ? tets[s] : faces[s - 4 * T]);
    slot[s] = (uint32_t)s;
}

__global__ void k3m_lumped(const uint32_t *__restrict__ off, const uint32_t *__restrict__ slot, int64_t N, int64_t T,
                           const double *__restrict__ tg, double *__restrict__ ell)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    double a = 0.0;
    for (uint32_t k = off[i]; k < off[i + 1]; ++k) {
        const uint32_t s = slot[k];
        if (s < 4 * T) a += tg[12 * T + s / 4] / 4.0;
    }
    ell[i] = a;
}

// q = C M: rho_T = -div M_h at the 4 volume points of T, sigma = M_h . n at the 3 points of
// each boundary face.  One thread per tetrahedron or face.
__global__ void k3m_charges(const double *__restrict__ M, const int32_t *__restrict__ tets, int64_t T,
                            const int32_t *__restrict__ faces, int64_t F, const double *__restrict__ tg,
                            const double *__restrict__ fg, double *__restrict__ q)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < T) {
        const int64_t t = k;
        double div = 0.0;
        for (int c = 0; c < 4; ++c) {
            const int64_t i = tets[4 * t + c];
            div += (M[3 * i] * tg[(3 * c) * T + t] + M[3 * i + 1] * tg[(3 * c + 1) * T + t]) +
                   M[3 * i + 2] * tg[(3 * c + 2) * T + t];
        }
        for (int c = 0; c < 4; ++c) q[4 * t + c] = -div;
    } else if (k < T + F) {
        const int64_t f = k - T;
        const double n0 = fg[0 * F + f], n1 = fg[1 * F + f], n2 = fg[2 * F + f];
        for (int qq = 0; qq < 3; ++qq) {
            double m[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < 3; ++c) {
                const int64_t i = faces[3 * f + c];
                const double l = c == qq ? FHI : FLO;
                for (int d = 0; d < 3; ++d) m[d] += l * M[3 * i + d];
            }
            q[4 * T + 3 * f + qq] = (m[0] * n0 + m[1] * n1) + m[2] * n2;
        }
    }
}

// out_i = (C^T u)_i, or with GRAD: out_i = -1/2 (l_i H_i + (C^T u)_i).
template <bool GRAD>
__global__ void k3m_charges_T(const uint32_t *__restrict__ off, const uint32_t *__restrict__ slot, int64_t N, int64_t T,
                              int64_t F, const double *__restrict__ tg, const double *__restrict__ fg,
                              const double *__restrict__ u, const double *__restrict__ ell, const double *__restrict__ H,
                              double *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    double o[3] = {0.0, 0.0, 0.0};
    for (uint32_t k = off[i]; k < off[i + 1]; ++k) {
        const int64_t s = slot[k];
        if (s < 4 * T) {
            const int64_t t = s / 4;
            const int c = (int)(s - 4 * t);
            const double us = ((u[4 * t] + u[4 * t + 1]) + u[4 * t + 2]) + u[4 * t + 3];
            for (int d = 0; d < 3; ++d) o[d] -= us * tg[(3 * c + d) * T + t];
        } else {
            const int64_t r = s - 4 * T, f = r / 3;
            const int c = (int)(r - 3 * f);
            double a = 0.0;
            for (int qq = 0; qq < 3; ++qq) a += (qq == c ? FHI : FLO) * u[4 * T + 3 * f + qq];
            for (int d = 0; d < 3; ++d) o[d] += a * fg[d * F + f];
        }
    }
    for (int d = 0; d < 3; ++d) out[3 * i + d] = GRAD ? -0.5 * (ell[i] * H[3 * i + d] + o[d]) : o[d];
}

// e_i = l_i M_i . H_i and V_i = l_i M_i
__global__ void k3m_energy_terms(const double *__restrict__ M, const double *__restrict__ H,
                                 const double *__restrict__ ell, int64_t N, double *__restrict__ e, double *__restrict__ V)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double l = ell[i];
    e[i] = l * ((M[3 * i] * H[3 * i] + M[3 * i + 1] * H[3 * i + 1]) + M[3 * i + 2] * H[3 * i + 2]);
    if (V)
        for (int d = 0; d < 3; ++d) V[3 * i + d] = l * M[3 * i + d];
}

__global__ void k3m_half_neg(const double *__restrict__ sum, double *__restrict__ E)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *E = -0.5 * sum[0];
}

struct MeshBuf3 {
    double *nodes = nullptr, *tg = nullptr, *fg = nullptr, *ell = nullptr, *x = nullptr, *w = nullptr;
    double *q = nullptr, *H = nullptr, *V = nullptr, *u = nullptr, *e = nullptr, *red = nullptr;
    int32_t *tets = nullptr, *faces = nullptr;
    uint32_t *off = nullptr, *slot = nullptr, *key = nullptr, *skey = nullptr, *sval = nullptr, *hist = nullptr;
};

}  // namespace fn3m

using namespace fn3m;

struct fn3_mesh {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t N = 0, T = 0, F = 0, S = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    MeshBuf3 b;
    bool ready = false;
    uint64_t stamp = 0;
    // binding (fn3_bind_mesh): the context, its geometry generation and this mesh's stamp then
    const fn3_ctx *bound = nullptr;
    uint64_t bound_gen = 0, bound_stamp = 0;
    std::string err;
};

namespace {

size_t mesh3_layout(const fn3_mesh *m, MeshBuf3 *b, char *base)
{
    const int64_t N = std::max<int64_t>(m->N, 1), T = std::max<int64_t>(m->T, 1), F = std::max<int64_t>(m->F, 1);
    const int64_t S = 4 * T + 3 * F;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = (o + bytes + 255) & ~(size_t)255;
        return base ? base + r : nullptr;
    };
    MeshBuf3 t;
    t.nodes = (double *)take(24 * N);
    t.tets = (int32_t *)take(16 * T);
    t.faces = (int32_t *)take(12 * F);
    t.tg = (double *)take(13 * 8 * T);
    t.fg = (double *)take(4 * 8 * F);
    t.ell = (double *)take(8 * N);
    t.off = (uint32_t *)take(4 * (N + 1));
    t.slot = (uint32_t *)take(4 * S);
    t.key = (uint32_t *)take(4 * S);
    t.skey = (uint32_t *)take(4 * S);
    t.sval = (uint32_t *)take(4 * S);
    t.hist = (uint32_t *)take(4 * 256 * ((S + 4095) / 4096));
    t.x = (double *)take(24 * S);
    t.w = (double *)take(8 * S);
    t.q = (double *)take(8 * S);
    t.u = (double *)take(8 * S);
    t.H = (double *)take(24 * N);
    t.V = (double *)take(24 * N);
    t.e = (double *)take(8 * N);
    t.red = (double *)take(8 * MESH_RED);
    if (b) *b = t;
    return o;
}

#define M3_ERR(mh, code, msg) \
    do {                      \
        (mh)->err = (msg);    \
        return (code);        \
    } while (0)

#define M3_HIP(mh, call)                                                                         \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            (mh)->err = std::string("HIP error in ") + #call + ": " + hipGetErrorString(e_);     \
            return FN_E_DEVICE;                                                                  \
        }                                                                                        \
    } while (0)

thread_local std::string g_mesh3_create_err;

int mesh3_select_device(fn3_mesh *m)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) M3_ERR(m, FN_E_DEVICE, std::string("pending HIP error: ") + hipGetErrorString(e));
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != m->device)
        if (hipSetDevice(m->device) != hipSuccess) M3_ERR(m, FN_E_DEVICE, "cannot select the mesh's device");
    return FN_OK;
}

int read_bad3(fn3_mesh *m, const double *part, int nblk, double *out)
{
    std::vector<double> h(nblk);
    M3_HIP(m, hipMemcpyAsync(h.data(), part, sizeof(double) * nblk, hipMemcpyDeviceToHost, m->stream));
    M3_HIP(m, hipStreamSynchronize(m->stream));
    double s = 0.0;
    for (double v : h) s += v;
    *out = s;
    return FN_OK;
}

// a failed call on the 3D context: its message becomes the mesh's
int ctx_fail(fn3_mesh *m, const fn3_ctx *ctx, int rc)
{
    const char *e = fn3_last_error(ctx);
    m->err = std::string("3D context: ") + (e ? e : "");
    return rc;
}

int mesh3_ready(fn3_mesh *m)
{
    if (!m->ready) M3_ERR(m, FN_E_STATE, "fn3_mesh_set must succeed first");
    return mesh3_select_device(m);
}

}  // namespace

extern "C" {

int fn3_mesh_create(int64_t n_nodes, int64_t n_tets, int64_t n_bfaces, void *stream, fn3_mesh **out)
{
    if (!out) { g_mesh3_create_err = "out is NULL"; return FN_E_INVAL; }
    *out = nullptr;
    if (n_nodes < 4 || n_tets < 1 || n_bfaces < 0 || n_nodes >= ((int64_t)1 << 31) ||
        4 * n_tets + 3 * n_bfaces >= ((int64_t)1 << 31)) {
        g_mesh3_create_err = "need n_nodes >= 4, n_tets >= 1, n_bfaces >= 0, nodes and 4 n_tets + 3 n_bfaces < 2^31";
        return FN_E_INVAL;
    }
    fn3_mesh *m = new (std::nothrow) fn3_mesh();
    if (!m) { g_mesh3_create_err = "out of host memory"; return FN_E_NOMEM; }
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        g_mesh3_create_err = "no HIP device";
        return FN_E_DEVICE;
    }
    m->stream = static_cast<hipStream_t>(stream);
    m->N = n_nodes;
    m->T = n_tets;
    m->F = n_bfaces;
    m->S = 4 * n_tets + 3 * n_bfaces;
    *out = m;
    return FN_OK;
}

int fn3_mesh_destroy(fn3_mesh *mesh)
{
    delete mesh;
    return FN_OK;
}

int fn3_mesh_workspace_size(const fn3_mesh *mesh, size_t *bytes)
{
    if (!mesh || !bytes) return FN_E_INVAL;
    *bytes = mesh3_layout(mesh, nullptr, nullptr);
    return FN_OK;
}

int fn3_mesh_set_workspace(fn3_mesh *mesh, void *dev_ptr, size_t bytes)
{
    if (!mesh) return FN_E_INVAL;
    if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255))
        M3_ERR(mesh, FN_E_INVAL, "workspace must be non-NULL and 256-byte aligned");
    if (bytes < mesh3_layout(mesh, nullptr, nullptr)) M3_ERR(mesh, FN_E_NOMEM, "mesh workspace too small");
    mesh->ws = dev_ptr;
    mesh->ws_bytes = bytes;
    mesh3_layout(mesh, &mesh->b, static_cast<char *>(dev_ptr));
    mesh->ready = false;
    return FN_OK;
}

int fn3_mesh_set(fn3_mesh *mesh, const double *nodes, const int32_t *tets, const int32_t *bfaces)
{
    if (!mesh) return FN_E_INVAL;
    fn3_mesh *m = mesh;
    if (!m->ws) M3_ERR(m, FN_E_STATE, "fn3_mesh_set_workspace must be called before fn3_mesh_set");
    if (!nodes || !tets || (m->F > 0 && !bfaces)) M3_ERR(m, FN_E_INVAL, "NULL mesh array");
    if (stream_capturing(m->stream)) M3_ERR(m, FN_E_STATE, "fn3_mesh_set waits for the device: not during graph capture");
    int rc = mesh3_select_device(m);
    if (rc) return rc;
    m->ready = false;
    const MeshBuf3 &b = m->b;
    hipStream_t st = m->stream;
    M3_HIP(m, hipMemcpyAsync(b.nodes, nodes, 24 * m->N, hipMemcpyDeviceToDevice, st));
    M3_HIP(m, hipMemcpyAsync(b.tets, tets, 16 * m->T, hipMemcpyDeviceToDevice, st));
    if (m->F > 0) M3_HIP(m, hipMemcpyAsync(b.faces, bfaces, 12 * m->F, hipMemcpyDeviceToDevice, st));
    const int nv = nb_grid(std::max<int64_t>(3 * m->N, std::max<int64_t>(4 * m->T, 3 * m->F)));
    k3m_validate<<<nv, FB, 0, st>>>(b.nodes, m->N, b.tets, m->T, b.faces, m->F, b.red);
    M3_HIP(m, hipGetLastError());
    double bad = 0.0;
    rc = read_bad3(m, b.red, nv, &bad);
    if (rc) return rc;
    if (bad > 0.0) M3_ERR(m, FN_E_INVAL, "vertex index out of range or non-finite node coordinate");
    const int nt = nb_grid(m->T), nf = nb_grid(m->F);
    k3m_tet_geom<<<nt, FB, 0, st>>>(b.nodes, b.tets, m->T, b.tg, b.red);
    k3m_face_geom<<<nf, FB, 0, st>>>(b.nodes, b.faces, m->F, b.fg, b.red + 256);
    M3_HIP(m, hipGetLastError());
    double bad_t = 0.0, bad_f = 0.0;
    rc = read_bad3(m, b.red, nt, &bad_t);
    if (rc) return rc;
    if (m->F > 0) {
        rc = read_bad3(m, b.red + 256, nf, &bad_f);
        if (rc) return rc;
    }
    if (bad_t > 0.0) M3_ERR(m, FN_E_DOMAIN, "degenerate tetrahedron (zero volume)");
    if (bad_f > 0.0) M3_ERR(m, FN_E_DOMAIN, "degenerate boundary face (zero area)");
    k3m_inc_keys<<<nb_of(m->S), FB, 0, st>>>(b.tets, m->T, b.faces, m->F, b.key, b.slot);
    M3_HIP(m, hipGetLastError());
    int keybits = 1;
    while (((int64_t)1 << keybits) < m->N) ++keybits;
    M3_HIP(m, fn::radix_sort(b.key, b.slot, b.skey, b.sval, b.hist, m->S, keybits, st));
    M3_HIP(m, fn::launch_cellstart(b.key, m->S, m->N, b.off, st));
    k3m_lumped<<<nb_of(m->N), FB, 0, st>>>(b.off, b.slot, m->N, m->T, b.tg, b.ell);
    k3m_sources<<<nb_of(m->S), FB, 0, st>>>(b.nodes, b.tets, m->T, b.faces, m->F, b.tg, b.fg, b.x, b.w);
    M3_HIP(m, hipGetLastError());
    M3_HIP(m, hipStreamSynchronize(st));
    m->ready = true;
    m->stamp++;
    return FN_OK;
}

int fn3_mesh_sources(fn3_mesh *mesh, double *x, double *w)
{
    if (!mesh) return FN_E_INVAL;
    int rc = mesh3_ready(mesh);
    if (rc) return rc;
    if (!x && !w) M3_ERR(mesh, FN_E_INVAL, "both outputs are NULL");
    if (x) M3_HIP(mesh, hipMemcpyAsync(x, mesh->b.x, 24 * mesh->S, hipMemcpyDeviceToDevice, mesh->stream));
    if (w) M3_HIP(mesh, hipMemcpyAsync(w, mesh->b.w, 8 * mesh->S, hipMemcpyDeviceToDevice, mesh->stream));
    return FN_OK;
}

int fn3_mesh_lumped_mass(fn3_mesh *mesh, double *ell)
{
    if (!mesh) return FN_E_INVAL;
    int rc = mesh3_ready(mesh);
    if (rc) return rc;
    if (!ell) M3_ERR(mesh, FN_E_INVAL, "ell is NULL");
    M3_HIP(mesh, hipMemcpyAsync(ell, mesh->b.ell, 8 * mesh->N, hipMemcpyDeviceToDevice, mesh->stream));
    return FN_OK;
}

int fn3_mesh_charges(fn3_mesh *mesh, const double *M, double *q)
{
    if (!mesh) return FN_E_INVAL;
    int rc = mesh3_ready(mesh);
    if (rc) return rc;
    if (!M || !q) M3_ERR(mesh, FN_E_INVAL, "NULL M or q");
    const MeshBuf3 &b = mesh->b;
    k3m_charges<<<nb_of(mesh->T + mesh->F), FB, 0, mesh->stream>>>(M, b.tets, mesh->T, b.faces, mesh->F, b.tg, b.fg, q);
    M3_HIP(mesh, hipGetLastError());
    return FN_OK;
}

int fn3_mesh_charges_T(fn3_mesh *mesh, const double *u, double *out)
{
    if (!mesh) return FN_E_INVAL;
    int rc = mesh3_ready(mesh);
    if (rc) return rc;
    if (!u || !out) M3_ERR(mesh, FN_E_INVAL, "NULL u or out");
    const MeshBuf3 &b = mesh->b;
    k3m_charges_T<false><<<nb_of(mesh->N), FB, 0, mesh->stream>>>(b.off, b.slot, mesh->N, mesh->T, mesh->F, b.tg, b.fg,
                                                                 u, nullptr, nullptr, out);
    M3_HIP(mesh, hipGetLastError());
    return FN_OK;
}

int fn3_bind_mesh(fn3_ctx *ctx, fn3_mesh *mesh)
{
    if (!ctx || !mesh) return FN_E_INVAL;
    if (!mesh->ready) M3_ERR(mesh, FN_E_STATE, "fn3_mesh_set must succeed before fn3_bind_mesh");
    if (mesh->device != fn3_internal_device(ctx)) M3_ERR(mesh, FN_E_INVAL, "mesh and context live on different devices");
    mesh->bound = nullptr;
    const int rc = fn3_set_geometry(ctx, mesh->N, mesh->b.nodes, mesh->S, mesh->b.x, mesh->b.w);
    if (rc) return ctx_fail(mesh, ctx, rc);
    mesh->bound = ctx;
    mesh->bound_gen = fn3_internal_geom_gen(ctx);
    mesh->bound_stamp = mesh->stamp;
    return FN_OK;
}

int fn3_energy(fn3_ctx *ctx, fn3_mesh *mesh, const double *M, double *E, double *grad)
{
    if (!ctx || !mesh) return FN_E_INVAL;
    if (!M || !E) M3_ERR(mesh, FN_E_INVAL, "NULL M or E");
    if (mesh->bound != ctx || mesh->bound_gen != fn3_internal_geom_gen(ctx) || mesh->bound_stamp != mesh->stamp ||
        !mesh->ready)
        M3_ERR(mesh, FN_E_STATE, "fn3_bind_mesh(ctx, mesh) must succeed after the last fn3_mesh_set and fn3_set_geometry");
    int rc = mesh3_select_device(mesh);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(fn3_internal_stream(ctx));
    const MeshBuf3 &b = mesh->b;
    k3m_charges<<<nb_of(mesh->T + mesh->F), FB, 0, st>>>(M, b.tets, mesh->T, b.faces, mesh->F, b.tg, b.fg, b.q);
    M3_HIP(mesh, hipGetLastError());
    rc = fn3_set_charges(ctx, b.q);
    if (rc) return ctx_fail(mesh, ctx, rc);
    rc = fn3_eval(ctx, nullptr, b.H);
    if (rc) return ctx_fail(mesh, ctx, rc);
    k3m_energy_terms<<<nb_of(mesh->N), FB, 0, st>>>(M, b.H, b.ell, mesh->N, b.e, b.V);
    M3_HIP(mesh, hipGetLastError());
    M3_HIP(mesh, fn::launch_sum(b.e, mesh->N, b.red, st));
    k3m_half_neg<<<1, 64, 0, st>>>(b.red, E);
    M3_HIP(mesh, hipGetLastError());
    if (!grad) return FN_OK;
    rc = fn3_eval_H_adjoint(ctx, b.V, b.u);
    if (rc) return ctx_fail(mesh, ctx, rc);
    k3m_charges_T<true><<<nb_of(mesh->N), FB, 0, st>>>(b.off, b.slot, mesh->N, mesh->T, mesh->F, b.tg, b.fg, b.u,
                                                       b.ell, b.H, grad);
    M3_HIP(mesh, hipGetLastError());
    return FN_OK;
}

const char *fn3_mesh_last_error(const fn3_mesh *mesh)
{
    if (!mesh) return g_mesh3_create_err.c_str();
    return mesh->err.c_str();
}

}  // extern "C"
