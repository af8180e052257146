/*
 * femnfft -- NFFT fast summation of 2D magnetostatic potentials and fields on MI355X.
 *
 * Operation (Kritsikis, Toussaint, Fruchart, "Fast computation of magnetostatic
 * fields by Non-uniform Fast Fourier Transforms"): for targets r_i (mesh nodes)
 * and sources r_j (quadrature points) of weight w_j = omega_j det J(r_j) carrying
 * a charge density q_j (volume rho_j or surface sigma_j), the discrete Green sum
 * of the paper's eq. (2)
 *
 *     phi_i = sum_j w_j q_j G(r_i - r_j),         G(r) = -(1/2 pi) ln |r|
 *
 * (G is the 2D Green function given with eq. (1)) and the field H = -grad phi
 * (introduction):
 *
 *     H_i   = (1/2 pi) sum_j w_j q_j (r_i - r_j) / |r_i - r_j|^2.
 *
 * Pairs at distance zero contribute nothing.  The sums are evaluated in
 * O(N log N) by the NFFT method of the paper's "NFFT" section: spread onto an
 * oversampled grid with a Kaiser-Bessel window, 2D FFT, multiply by the Fourier
 * coefficients of the kernel smoothed near the origin (window deconvolution
 * folded into the same table), inverse FFT, gather at the targets, plus a
 * near-field correction in the smoothing zone.  The transposes (adjoints) of
 * both maps with respect to q are provided for gradients.
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer on the device that was current
 *     at fn_create, unless stated otherwise.  The caller owns all of them.
 *   - 2-vectors are interleaved [n][2] (x, y), FP64.  Scalars per point FP64.
 *   - All work is enqueued on the stream given to fn_create; no call waits for
 *     the device except fn_set_geometry (it reads back the bounding box) and
 *     fn_mesh_set.  Outputs are valid once the stream reaches them.
 *   - The library allocates no device memory after fn_set_workspace: the caller
 *     provides one workspace buffer (e.g. a torch uint8 tensor).
 *   - Call order per context: fn_create -> fn_workspace_size -> fn_set_workspace
 *     -> fn_set_geometry -> fn_set_charges -> fn_eval*; fn_eval_*_adjoint only
 *     needs fn_set_geometry.  Out-of-order calls return FN_E_STATE.
 *   - A context is not thread-safe; use one context per stream.
 *   - Every function returns FN_OK (0) or an FN_E_* code; fn_last_error()
 *     gives a message.  No C++ exception crosses this interface.
 *   - Debug checks: with the environment variable FEMNFFT_DEBUG_CHECKS set to a
 *     value other than "0" when fn_create / fn3_create runs, fn_set_geometry and
 *     fn3_set_geometry validate every binned point set on the device (keys sorted
 *     and inside the cell table, cell starts consistent with the keys, cell
 *     fractions in [0, 1] in 2D, packed positions inside their key's cell in 3D,
 *     the sort permutation a permutation) and return FN_E_DEVICE with the count of
 *     violations in the message.  The checks wait for the stream; results are the
 *     same bit for bit with and without them.
 */
#ifndef FEMNFFT_H
#define FEMNFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FN_OK = 0,
    FN_E_INVAL = 1,       /* null pointer, bad size or parameter, non-finite input */
    FN_E_STATE = 2,       /* call out of order */
    FN_E_DOMAIN = 3,      /* degenerate geometry (all points coincide) */
    FN_E_NOMEM = 4,       /* workspace too small */
    FN_E_DEVICE = 5,      /* HIP runtime error (includes asynchronous faults) */
    FN_E_UNSUPPORTED = 6  /* parameter combination not implemented */
};

enum {
    FN_FP64 = 0,       /* spread, FFT, gather, near field all in FP64 */
    FN_FP32_MIXED = 1  /* FP32 spread/FFT/gather (wide accumulation); near field FP64 except its
                          per-pair ln x and 1/x (FP32 hardware instructions); FP64 final sum */
};

/*
 * Parameters of the method (all lengths on the unit torus the points are mapped to).
 *   grid      G, the oversampled FFT grid per dimension; power of two, 64..8192.
 *   m         Kaiser-Bessel half-width in grid cells (2m taps per dimension), 2..8.
 *   p         regularization degree: the kernel is replaced near the origin by an
 *             even polynomial matching ln r and its first p-1 derivatives at eps_I
 *             (the paper's "smoothness degree"), 1..12.
 *   eps_I     near-field radius; 0 < eps_I, eps_I * G <= 32.
 *   eps_B     width of the boundary regularization near |x| = 1/2; 0 < eps_B < 1/4.
 *   precision FN_FP64 or FN_FP32_MIXED.
 *   n         bandwidth; the window shape is b = pi (2 - 1/sigma), sigma = G/n.
 *   eps_S     near-field radius of surface sources (fn_set_geometry_split), 0 or in
 *             the range of eps_I.  The sum is linear in the sources, so each class can
 *             be summed with its own regularized kernel: the surface (line) charges
 *             with K_R at eps_S, the others with K_R at eps_I.  Line charges need the
 *             larger radius -- the error of the truncated Fourier series of K_R
 *             concentrates near |r| = eps_I, where a line tangent to that circle sums
 *             it up while an area density averages it out -- so eps_I can then be set
 *             for the volume charges alone.  0: every source uses eps_I.
 */
typedef struct fn_params {
    int32_t grid;
    int32_t m;
    int32_t p;
    int32_t precision;
    double eps_I;
    double eps_B;
    int32_t flags;      /* reserved, must be 0 */
    int32_t n;          /* bandwidth (kept Fourier modes |l| <= n/2): 0 means G/2 (oversampling
                           2); otherwise even, G/2 <= n <= 3G/4, a power of two or three
                           times one (3G/4: oversampling 4/3) */
    double eps_S;       /* near-field radius of the surface sources; 0: none (see above) */
} fn_params;

/* Read-only facts about a context after fn_set_geometry (host struct). */
typedef struct fn_info {
    double centre[2];       /* c: bounding-box midpoint of all points */
    double scale;           /* s: torus coordinate = s (r - c) */
    int64_t n_tgt, n_src;
    int32_t win_lo[2];      /* first grid index (x, y) of the data window */
    int32_t win_ext[2];     /* window extent in cells (x, y) */
    int32_t tiles[2];       /* spread/gather tiles per dimension */
    int32_t near_cells;     /* near-field radius in grid cells (ceil) */
    size_t workspace_bytes; /* bytes required for (n_tgt, n_src) */
    int64_t near_pairs;     /* (target, source) pairs closer than eps_I; with surface sources,
                               (target, volume source) pairs only */
    int64_t n_surf;         /* surface sources (the last n_surf sources), 0 without eps_S */
    int64_t near_pairs_surf;/* (target, surface source) pairs closer than eps_S */
    int32_t near_cells_surf;/* eps_S in grid cells (ceil) */
    int32_t reserved;
} fn_info;

typedef struct fn_ctx fn_ctx;

/* Fill *p with defaults for grid G: m = 6, p = 8, eps_I = 7/(G/2), eps_B = 1/16,
 * precision FN_FP32_MIXED. */
int fn_params_default(fn_params *p, int32_t grid);

/* Parameters for n_tgt targets and n_src sources at the accuracy the library is
 * tuned for (relative L2 error of phi, H and the adjoints ~1e-7 against the
 * exact sum on FEM meshes): m = 6, bandwidth n = 3G/4 (oversampling 4/3; G/2 for
 * G = 64), eps_I = 7/n, and p = 8 with G = 2^ceil(log2(sqrt(2 N))), N = n_tgt + n_src
 * -- or, below 2^22 points in total, where the boundary-layer error of H is a larger
 * share, p = 9 with G = 2^ceil(log2(sqrt(4 N))) (the larger grid keeps the near field
 * cheaper); G clamped to 64..8192. */
int fn_params_auto(int64_t n_tgt, int64_t n_src, int32_t precision, fn_params *p);

/* Create a context bound to the current device and to the HIP stream
 * `stream` (hipStream_t, may be NULL for the null stream).  Validates the
 * parameters and prepares the host-side plan (regularization polynomials,
 * window transform).  *out receives the context; free it with fn_destroy. */
int fn_create(const fn_params *params, void *stream, fn_ctx **out);
int fn_destroy(fn_ctx *ctx);

/* Bytes of device workspace needed for n_tgt targets and n_src sources
 * (an upper bound that does not depend on where the points lie). */
int fn_workspace_size(const fn_ctx *ctx, int64_t n_tgt, int64_t n_src, size_t *bytes);

/* Hand the context a device buffer of `bytes` bytes, 256-byte aligned.  The
 * context uses it until fn_destroy or the next fn_set_workspace; the caller must
 * keep it alive that long.  Builds the kernel's Fourier table (b_l and the
 * deconvolution) inside it. */
int fn_set_workspace(fn_ctx *ctx, void *dev_ptr, size_t bytes);

/* Targets tgt_xy [n_tgt][2], sources src_xy [n_src][2] with weights src_w [n_src]
 * (w_j = omega_j det J(r_j) of eq. (2)).  Maps all points to the unit torus
 * (centre c = bounding-box midpoint, D = 2 max |r - c|, s = (1/2 - eps_B)/D),
 * bins them by grid cell and keeps sorted copies in the workspace.  The input
 * buffers are not referenced after the call.  Blocks until the bounding box is
 * known.  FN_E_DOMAIN if every point coincides; FN_E_NOMEM if the workspace is
 * smaller than fn_workspace_size(n_tgt, n_src). */
int fn_set_geometry(fn_ctx *ctx, int64_t n_tgt, const double *tgt_xy,
                    int64_t n_src, const double *src_xy, const double *src_w);

/* As fn_set_geometry, with the last n_surf sources (0 <= n_surf <= n_src) marked as
 * surface quadrature points (boundary-edge points of the charge density sigma of eq.
 * (2)).  With eps_S > 0 they are summed with the kernel regularized at eps_S and
 * near-field radius eps_S, the other n_src - n_surf with eps_I; with eps_S = 0 the
 * call is fn_set_geometry.  The result is the sum of the two fast summations.
 * Order of the sources, weights, charges and adjoint outputs is unchanged. */
int fn_set_geometry_split(fn_ctx *ctx, int64_t n_tgt, const double *tgt_xy, int64_t n_src,
                          const double *src_xy, const double *src_w, int64_t n_surf);

/* Charge densities q [n_src] (rho_j or sigma_j of eq. (2)); copied into the
 * workspace as s_j = w_j q_j in binned order. */
int fn_set_charges(fn_ctx *ctx, const double *q);

/* phi [n_tgt] and/or H [n_tgt][2] at the targets; either pointer may be NULL
 * in fn_eval (not both, unless n_tgt is 0: then nothing is written and any
 * output may be NULL).  Results in the caller's target order. */
int fn_eval(fn_ctx *ctx, double *phi, double *H);
int fn_eval_phi(fn_ctx *ctx, double *phi);
int fn_eval_H(fn_ctx *ctx, double *H);

/* Transposes with respect to q (need fn_set_geometry only):
 *   fn_eval_phi_adjoint:  u_j = w_j sum_i v_i G(r_i - r_j)          v [n_tgt], u [n_src]
 *   fn_eval_H_adjoint:    u_j = w_j sum_i V_i . (-grad G)(r_i - r_j)
 *                             = w_j sum_i V_i . (r_i - r_j) / (2 pi |r_i - r_j|^2)
 *                                                                    V [n_tgt][2], u [n_src]
 * so that <H(q), V> = <q, u> and <phi(q), v> = <q, u> up to rounding. */
int fn_eval_phi_adjoint(fn_ctx *ctx, const double *v, double *u);
int fn_eval_H_adjoint(fn_ctx *ctx, const double *V, double *u);

/* phi of eq. (2) with H = -grad phi at the targets, and the transpose of the H map
 * applied to V: fn_eval(ctx, phi, H) and fn_eval_H_adjoint(ctx, V, u) in one call, the
 * two running at the same time (the pair a gradient of the demagnetizing energy needs): the adjoint on a second stream the context owns (created on the first
 * call, default priority, freed by fn_destroy), forked from and joined back into the
 * context's stream with events, so the call is ordered like the two calls on that stream
 * and can be captured into a graph once it has run once (FN_E_STATE if the first call is
 * made under capture).  Each direction has its own far-field scratch in the workspace;
 * one direction's kernels take the CUs the other leaves free.  Arguments as for the two
 * calls (phi or H may be NULL, not both unless n_tgt is 0; V [n_tgt][2], u [n_src]); the
 * outputs are written concurrently and must not overlap each other or the inputs.
 * Results equal those of the two calls (every kernel sums in a fixed order). */
int fn_eval_with_H_adjoint(fn_ctx *ctx, double *phi, double *H, const double *V, double *u);

int fn_get_info(const fn_ctx *ctx, fn_info *info);

/* Work shapes of the kernels: the knobs of the autotuner (paper_0807_2387_amd.tune), which
 * times candidates on the caller's own data and keeps the fastest per (grid, window, degree,
 * precision, points per cell, GPU architecture).  They change speed only; results change at
 * most by rounding (a different summation order).  A 0 field keeps the library default.
 *   spread_groups   FP32 spread: the 2m x 2m footprint of a cell's points is summed in
 *                   registers in this many groups of whole row pairs (1..3; at most 144
 *                   sums per group); default 1 for m <= 4, 2 for m <= 6, else 3.
 *   near_*_bx, _by  near-field home block of the volume sources, cells: 16 x 16, 32 x 8 or
 *                   64 x 4 (default 32 x 8), forward (targets home) and adjoint (sources home)
 *   near_*_cap      points of the other set staged per LDS chunk, a multiple of 64 in
 *                   [128, 2048] (default 1024 forward, 512 adjoint)
 *   tile            spread and gather tile edge, cells: 16 or 32 (default 32); smaller tiles
 *                   give small grids more workgroups
 * FN_E_INVAL for an unsupported value (nothing is changed then). */
typedef struct fn_shapes {
    int32_t spread_groups;
    int32_t near_fwd_bx, near_fwd_by, near_fwd_cap;
    int32_t near_adj_bx, near_adj_by, near_adj_cap;
    int32_t tile;
} fn_shapes;
int fn_set_shapes(fn_ctx *ctx, const fn_shapes *shapes);
int fn_get_shapes(const fn_ctx *ctx, fn_shapes *shapes);   /* the shapes in effect */

/* For callers that cannot allocate device memory (code under graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): fn_set_geometry_split + fn_set_charges + fn_eval
 * in one call whose workspace is a library-owned static device buffer of
 * FN_NOALLOC_SCRATCH_BYTES (64 MiB) per device, held from the library's load until the
 * process ends, instead of the context's own workspace.  The call allocates nothing
 * (no hipMalloc, no torch allocation); the caller passes the inputs and outputs as for
 * those calls (device pointers; the last n_surf sources are surface sources).  Problems
 * whose fn_workspace_size exceeds FN_NOALLOC_SCRATCH_BYTES are rejected with FN_E_NOMEM
 * before anything is read or launched.  The context only lends its parameters and stream:
 * its own workspace, geometry and charges are as before the call (fn_set_workspace is not
 * needed).  Like fn_set_geometry it waits for the device (it reads back the bounding box),
 * so it cannot itself be captured.  Every call on one device shares the buffer and keeps
 * the previous call's contents (the plan tables are reused when the parameters match;
 * everything else is rewritten before it is read): calls on one device are serialized on
 * the host, but their kernels race if they run at once on different streams, so a caller
 * must order calls made on different streams itself.  Results equal those of the three
 * calls on a context with its own workspace. */
#define FN_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int fn_eval_noalloc(fn_ctx *ctx, int64_t n_tgt, const double *tgt_xy, int64_t n_src, const double *src_xy,
                    const double *src_w, int64_t n_surf, const double *q, double *phi, double *H);

/* Stage timing with HIP events recorded on the context's stream around every
 * kernel stage of fn_set_charges / fn_eval* / fn_eval_*_adjoint.
 * fn_set_profiling(ctx, 1) starts recording (and clears the totals);
 * fn_get_profile waits for the recorded events, adds their elapsed times to
 * the totals and copies them out (host struct); recording continues until
 * fn_set_profiling(ctx, 0).  At most 8192 stages are recorded between two
 * fn_get_profile calls (later ones are dropped and counted in `dropped`). */
enum {
    FN_ST_CHARGES = 0, FN_ST_SPREAD, FN_ST_FOLD, FN_ST_ROWS_FWD, FN_ST_COLS, FN_ST_ROWS_INV,
    FN_ST_GATHER, FN_ST_NEAR,
    FN_ST_A_VALUES, FN_ST_A_SPREAD, FN_ST_A_FOLD, FN_ST_A_ROWS_FWD, FN_ST_A_COLS, FN_ST_A_ROWS_INV,
    FN_ST_A_GATHER, FN_ST_A_NEAR,
    FN_ST_NEAR_SURF, FN_ST_A_NEAR_SURF,   /* near field of the surface sources (eps_S) */
    FN_NUM_STAGES
};
typedef struct fn_profile {
    double ms[FN_NUM_STAGES];     /* summed event time per stage */
    int64_t count[FN_NUM_STAGES]; /* launches recorded per stage */
    int64_t dropped;
} fn_profile;
int fn_set_profiling(fn_ctx *ctx, int enable);
int fn_get_profile(fn_ctx *ctx, fn_profile *out);

/* Message of the last error on this context (or of the last failed
 * fn_create when ctx is NULL).  Valid until the next call on the context. */
const char *fn_last_error(const fn_ctx *ctx);

/*
 * P1 finite-element front (the paper's "Discretization" section): a triangle
 * mesh with nodal magnetization M, the volume charge rho = -div M_h (constant per
 * triangle) and the surface charge sigma = M_h . n on the boundary, integrated by
 * a 3-point rule per triangle (barycentric (2/3, 1/6, 1/6) and permutations,
 * weight |T|/3) and 2-point Gauss-Legendre per boundary edge (weight |e|/2).
 * The paper's quadrature footnote is missing; this rule is the reading taken.
 *
 *   nodes   [n_nodes][2]  FP64
 *   tris    [n_tris][3]   int32 vertex indices (either orientation)
 *   bedges  [n_bedges][2] int32 boundary edges (a, b) with the domain on the left
 *           of a -> b (outer boundary counter-clockwise, holes clockwise);
 *           outward normal (b - a) rotated by -90 degrees.
 *
 * Sources: S = 3 n_tris + 2 n_bedges quadrature points, the 3 volume points of
 * triangle t at 3t + k (k-th point nearest vertex k), then the 2 surface points of
 * edge e at 3 n_tris + 2e + k (Gauss points 1/2 -+ 1/(2 sqrt 3) along a -> b).
 * The charge operator is q = C M [S] (rho on volume points, sigma on surface
 * points) and C^T its exact transpose (nodal 2-vectors).  The lumped mass is
 * l_i = sum over triangles at node i of |T|/3.
 *
 * A mesh object holds copies of the arrays (in a caller workspace, as for the
 * context) plus its geometry and a node -> incident slot list, so that C^T and l
 * are fixed-order gathers (bitwise reproducible).  Every array argument is a
 * device pointer; work runs on the mesh's stream, except inside fn_energy, which
 * uses the context's stream.  Calls that overlap on one mesh race.
 */
typedef struct fn_mesh fn_mesh;

/* n_nodes >= 3, n_tris >= 1, n_bedges >= 0 (sizes are fixed for the object). */
int fn_mesh_create(int64_t n_nodes, int64_t n_tris, int64_t n_bedges, void *stream, fn_mesh **out);
int fn_mesh_destroy(fn_mesh *mesh);
int fn_mesh_workspace_size(const fn_mesh *mesh, size_t *bytes);
int fn_mesh_set_workspace(fn_mesh *mesh, void *dev_ptr, size_t bytes);  /* 256-byte aligned */
/* Copy and check the mesh (indices in range, finite nodes: FN_E_INVAL; zero-area
 * triangles -- twice the area at most 1e-12 of |dx1 dy2| + |dy1 dx2| -- or
 * zero-length edges: FN_E_DOMAIN), build its geometry, sources,
 * lumped mass and incidence list.  Blocks until done. */
int fn_mesh_set(fn_mesh *mesh, const double *nodes, const int32_t *tris, const int32_t *bedges);
int fn_mesh_sources(fn_mesh *mesh, double *x, double *w);           /* x [S][2], w [S]; either may be NULL */
int fn_mesh_lumped_mass(fn_mesh *mesh, double *ell);                /* ell [n_nodes] */
int fn_mesh_charges(fn_mesh *mesh, const double *M, double *q);     /* M [n_nodes][2] -> q [S] */
int fn_mesh_charges_T(fn_mesh *mesh, const double *u, double *out); /* u [S] -> out [n_nodes][2] */

/* Use the mesh's nodes as targets and its quadrature points as sources of the
 * context (fn_set_geometry_split with them: the boundary-edge points are the
 * surface sources, which take eps_S when it is set). */
int fn_bind_mesh(fn_ctx *ctx, fn_mesh *mesh);

/* Demagnetizing energy of nodal magnetization M [n_nodes][2] and its gradient:
 *     H = fast-sum field at the nodes of q = C M,
 *     E = -1/2 sum_i l_i M_i . H_i                     -> *E (one device double)
 *     grad = dE/dM = -1/2 (l H + C^T u),  u = H-adjoint of V = l M
 *                                                      -> grad [n_nodes][2] (may be NULL)
 * Needs fn_bind_mesh(ctx, mesh) after the mesh's last fn_mesh_set.  Runs on the
 * context's stream; uses the mesh's scratch (q, H, V, u) and the context's
 * charges (a following fn_eval sees C M).  With grad, H and u are computed at once
 * as in fn_eval_with_H_adjoint (V needs only M), except under graph capture before
 * that call has created its stream: then one after the other. */
int fn_energy(fn_ctx *ctx, fn_mesh *mesh, const double *M, double *E, double *grad);

/* Outputs at the quadrature points (the Discretization section's charges sit there).
 * fn_bind_mesh_sources: the mesh's quadrature points are both the targets and the sources
 * of the context, all in one source class (every source takes the kernel regularized at
 * eps_I; eps_S is not used): the fast potential matrix is then symmetric like the exact
 * one.  The potential of eq. (2) at a point leaves that point's own charge out, like any
 * pair at distance 0.  The context's workspace must hold fn_workspace_size(S, S).
 * fn_energy_charge: with q = C M and s = w q,
 *     phi_j = sum_{k != j} s_k G(r_j - r_k)        -> phi_s [S] (may be NULL)
 *     E_q   = 1/2 sum_j s_j phi_j                   -> *E (one device double)
 *     grad  = dE_q/dM = C^T (w phi)                 -> grad [n_nodes][2] (may be NULL)
 * E_q is the energy of the charges in their own potential (1/2 int rho phi + 1/2 oint
 * sigma phi by the same quadrature, mu0 = 1).  The potential matrix between distinct
 * points is symmetric (the fast one too, with one source class), so the gradient needs no
 * adjoint evaluation.  Runs on the context's stream; needs fn_bind_mesh_sources(ctx,
 * mesh) after the last fn_mesh_set. */
int fn_bind_mesh_sources(fn_ctx *ctx, fn_mesh *mesh);
int fn_energy_charge(fn_ctx *ctx, fn_mesh *mesh, const double *M, double *E, double *grad, double *phi_s);

/* The field of the P1 interpolant of a nodal potential phi [n_nodes] (e.g. phi of eq. (2)
 * at the nodes): H_T = -sum_k phi_{i_k} grad(lambda_k) per triangle -> H_tri [n_tris][2],
 * and its lumped projection H_i = (1/l_i) sum_{T at i} (|T|/3) H_T -> H_node [n_nodes][2]
 * (either may be NULL, not both).  FP64, fixed summation order, on the mesh's stream. */
int fn_mesh_p1_gradient(fn_mesh *mesh, const double *phi, double *H_tri, double *H_node);

/* Message of the last error on this mesh (or of the last failed fn_mesh_create
 * when mesh is NULL). */
const char *fn_mesh_last_error(const fn_mesh *mesh);

/*
 * Batches: B independent problems (e.g. one per mesh) in one object, each with
 * its own parameters (typically its own grid).  Inputs and outputs are the members'
 * arrays concatenated; tgt_off / src_off are HOST arrays of B + 1 offsets
 * (0 = tgt_off[0] <= tgt_off[1] <= ...), in points.  Each member needs at least one
 * point.  Member b's targets are tgt_xy[tgt_off[b] .. tgt_off[b+1]) and so on; phi, H,
 * q, V, v, u likewise.  The workspace is one caller buffer carved into the members'
 * workspaces.  Every evaluation call is ordered on the batch stream; inside it the
 * members' tasks (forwards and adjoints) run over the batch's lanes: streams it owns
 * (default priority, created by the first evaluation or fn_batch_set_lanes, freed by
 * fn_batch_destroy), forked from the batch stream with one event and joined back, the
 * tasks given to the lanes longest first by a cost model (near-field pairs, points, grid
 * cells) so that small members' kernels run side by side.  A batch evaluation records
 * into one graph once the lanes exist (FN_E_STATE if the first evaluation is captured).
 * Evaluation arguments are checked for the whole batch before anything is enqueued.
 */
typedef struct fn_batch fn_batch;
int fn_batch_create(int32_t count, const fn_params *params /* [count] */, void *stream, fn_batch **out);
int fn_batch_destroy(fn_batch *batch);
int fn_batch_workspace_size(fn_batch *batch, const int64_t *tgt_off, const int64_t *src_off, size_t *bytes);
int fn_batch_set_workspace(fn_batch *batch, void *dev_ptr, size_t bytes);  /* 256-byte aligned */
int fn_set_geometry_batch(fn_batch *batch, const int64_t *tgt_off, const double *tgt_xy,
                          const int64_t *src_off, const double *src_xy, const double *src_w);
/* As fn_set_geometry_batch; member i's last n_surf[i] sources are surface sources
 * (fn_set_geometry_split).  n_surf [count] is a host array; NULL means none. */
int fn_set_geometry_batch_split(fn_batch *batch, const int64_t *tgt_off, const double *tgt_xy,
                                const int64_t *src_off, const double *src_xy, const double *src_w,
                                const int64_t *n_surf);
/* Number of lanes (streams) an evaluation spreads the members' tasks over, 1..8 (default
 * 4, the hardware queues a process gets by default); creates them now.  Not during capture. */
int fn_batch_set_lanes(fn_batch *batch, int32_t lanes);
int fn_batch_set_charges(fn_batch *batch, const double *q);
int fn_batch_eval(fn_batch *batch, double *phi, double *H);        /* either may be NULL, not both */
int fn_batch_eval_H_adjoint(fn_batch *batch, const double *V, double *u);
/* fn_batch_eval(batch, phi, H) and fn_batch_eval_H_adjoint(batch, V, u) in one call, as
 * fn_eval_with_H_adjoint does for one context (phi and H = -grad phi of eq. (2), and the
 * transpose of the H map): every member's forward and adjoint are tasks of one schedule
 * over the lanes (a member's two directions use separate scratch and may run at the same
 * time).  Outputs must not overlap each other or the inputs; results equal those of the
 * two calls. */
int fn_batch_eval_with_H_adjoint(fn_batch *batch, double *phi, double *H, const double *V, double *u);
int fn_batch_eval_phi_adjoint(fn_batch *batch, const double *v, double *u);
/* Borrow member i's context (owned by the batch: never destroy it, and call nothing on it
 * while a batch call runs).  fn_set_shapes / fn_get_shapes on it set or read that member's
 * kernel shapes for the following batch evaluations (the batch workspace fits every
 * supported shape); fn_get_info and fn_last_error read it.  Calls that change its
 * geometry, workspace or charges belong to the fn_batch_* functions. */
int fn_batch_member(fn_batch *batch, int32_t i, fn_ctx **out);
const char *fn_batch_last_error(const fn_batch *batch);

/*
 * Graph capture.  fn_graph_begin(stream) starts capturing (hipStreamCaptureModeThreadLocal)
 * the work this thread then issues on `stream` (non-NULL): fn_set_charges,
 * fn_eval*, fn_eval_*_adjoint, fn_energy, fn_mesh_charges(_T) and the fn_batch_*
 * evaluations record their kernels with the argument values and pointers of that
 * moment; fn_graph_end instantiates the graph; fn_graph_launch replays it (on any
 * stream), reading whatever the recorded input buffers hold then.  Calls that
 * wait for the device (fn_set_geometry, fn_mesh_set, fn_get_profile) return
 * FN_E_STATE during capture; stage profiling is not recorded inside graphs.  The
 * recorded contexts, meshes and buffers must outlive the graph, and replays of
 * one graph (or a replay and a direct call on the same context) must not overlap.
 */
typedef struct fn_graph fn_graph;
int fn_graph_begin(void *stream);
int fn_graph_end(void *stream, fn_graph **out);
int fn_graph_launch(fn_graph *graph, void *stream);
int fn_graph_destroy(fn_graph *graph);
const char *fn_graph_last_error(void);

/*
 * The same fast summation in 3D: eq. (2) with the 3D Green function given with eq. (1),
 *
 *     phi_i = sum_j w_j q_j / (4 pi |r_i - r_j|),
 *     H_i   = -grad phi = (1/4pi) sum_j w_j q_j (r_i - r_j) / |r_i - r_j|^3,
 *
 * and the transpose of the H map, u_j = w_j sum_i V_i . (r_i - r_j) / (4 pi |r_i - r_j|^3),
 * by the NFFT method on a G^3 grid (the paper's p^3 N grid in 3D), for tetrahedral FEM
 * quadrature points or any point sets.  FP64 throughout (precision must be FN_FP64), grid G
 * a power of two in [16, 256], m <= G/4 - 1, eps_S = 0; bandwidth n = 0 (G/2, oversampling 2)
 * or even in [G/2, 3G/4] (at n = 3G/4 the window needs m >= 5 for errors below 1e-7, and the
 * near radius eps_I shrinks with 1/n; FN_E_INVAL otherwise).  3-vectors are interleaved
 * [n][3]; every array is a device pointer; the conventions (ordering, workspace, call order,
 * errors, pairs at distance zero) are those of the 2D context.  The kernel's regularization
 * near the torus boundary needs a wider zone than in 2D: eps_B = 1/8 is the tested setting.
 */
typedef struct fn3_ctx fn3_ctx;
int fn3_create(const fn_params *params, void *stream, fn3_ctx **out);
int fn3_destroy(fn3_ctx *ctx);
int fn3_workspace_size(const fn3_ctx *ctx, int64_t n_tgt, int64_t n_src, size_t *bytes);
int fn3_set_workspace(fn3_ctx *ctx, void *dev_ptr, size_t bytes);
int fn3_set_geometry(fn3_ctx *ctx, int64_t n_tgt, const double *tgt_xyz, int64_t n_src, const double *src_xyz,
                     const double *src_w);
int fn3_set_charges(fn3_ctx *ctx, const double *q);
int fn3_eval(fn3_ctx *ctx, double *phi, double *H);                   /* phi [n_tgt], H [n_tgt][3] */
int fn3_eval_H_adjoint(fn3_ctx *ctx, const double *V, double *u);     /* V [n_tgt][3], u [n_src] */
/* facts after fn3_set_geometry (host outputs, any may be NULL): point counts, torus scale s,
 * data window extent [3] in cells, near radius in cells */
int fn3_get_info(const fn3_ctx *ctx, int64_t *n_tgt, int64_t *n_src, double *scale, int32_t *win_ext,
                 int32_t *near_cells);
/* Stage timing of the 3D context (the 2D context's fn_set_profiling / fn_get_profile
 * conventions; at most 4096 stages between two fn3_get_profile calls), filling the
 * first FN3_NUM_STAGES entries of an fn_profile with these stages: */
enum {
    FN3_ST_CHARGES = 0, FN3_ST_SPREAD, FN3_ST_FFT, FN3_ST_MULTIPLY, FN3_ST_IFFT, FN3_ST_GATHER, FN3_ST_NEAR,
    FN3_ST_A_VALUES, FN3_ST_A_SPREAD, FN3_ST_A_FFT, FN3_ST_A_MULTIPLY, FN3_ST_A_IFFT, FN3_ST_A_GATHER,
    FN3_ST_A_NEAR,
    FN3_NUM_STAGES
};
int fn3_set_profiling(fn3_ctx *ctx, int enable);

/*
 * 3D FEM front on tetrahedra (the 2D fn_mesh_* calls with tetrahedra and boundary
 * triangles; the Discretization section's P1 interpolation of M, rho = -div M and
 * sigma = M.n, quadrature points with weights omega_j det J):
 *   nodes [n_nodes][3] FP64, tets [n_tets][4] int32 (any orientation), bfaces [n_bfaces][3]
 *   int32 with (b - a) x (c - a) pointing out of the domain; M [n_nodes][3].
 * Sources (S = 4 n_tets + 3 n_bfaces): 4 points per tetrahedron at barycentric
 * (a, b, b, b) and permutations, a = (5 + 3 sqrt 5)/20, b = (5 - sqrt 5)/20, weight |T|/4,
 * then 3 points per boundary face at (2/3, 1/6, 1/6) and permutations, weight |F|/3.
 * q = C M: -div M_h at the volume points, M_h . n at the face points; C^T its transpose;
 * lumped mass l_i = sum |T|/4 over the tetrahedra at node i.  Workspace, stream, error
 * and ordering conventions are those of fn_mesh_*; fn3_mesh_set checks indices and
 * finiteness (FN_E_INVAL) and zero-volume tetrahedra (|det J| <= 1e-12 |e1||e2||e3|) or
 * zero-area faces (FN_E_DOMAIN), and blocks until done.
 * fn3_bind_mesh: the mesh's nodes become the targets and its quadrature points the
 * sources of the 3D context (fn3_set_geometry).
 * fn3_energy: E = -1/2 sum_i l_i M_i . H_i (one device double) and, if grad is not NULL,
 * dE/dM = -1/2 (l H + C^T A^T (l M)) [n_nodes][3], with H = A C M the 3D fast-sum field
 * at the nodes; on the context's stream; needs fn3_bind_mesh after the last fn3_mesh_set
 * and fn3_set_geometry (else FN_E_STATE).  fn3_bind_mesh and fn3_energy report every
 * error, the context's included, through fn3_mesh_last_error(mesh).
 */
typedef struct fn3_mesh fn3_mesh;
int fn3_mesh_create(int64_t n_nodes, int64_t n_tets, int64_t n_bfaces, void *stream, fn3_mesh **out);
int fn3_mesh_destroy(fn3_mesh *mesh);
int fn3_mesh_workspace_size(const fn3_mesh *mesh, size_t *bytes);
int fn3_mesh_set_workspace(fn3_mesh *mesh, void *dev_ptr, size_t bytes);
int fn3_mesh_set(fn3_mesh *mesh, const double *nodes, const int32_t *tets, const int32_t *bfaces);
int fn3_mesh_sources(fn3_mesh *mesh, double *x, double *w);          /* x [S][3], w [S]; either may be NULL */
int fn3_mesh_lumped_mass(fn3_mesh *mesh, double *ell);               /* ell [n_nodes] */
int fn3_mesh_charges(fn3_mesh *mesh, const double *M, double *q);    /* M [n_nodes][3] -> q [S] */
int fn3_mesh_charges_T(fn3_mesh *mesh, const double *u, double *out);/* u [S] -> out [n_nodes][3] */
int fn3_bind_mesh(fn3_ctx *ctx, fn3_mesh *mesh);
int fn3_energy(fn3_ctx *ctx, fn3_mesh *mesh, const double *M, double *E, double *grad);
const char *fn3_mesh_last_error(const fn3_mesh *mesh);
int fn3_get_profile(fn3_ctx *ctx, fn_profile *out);
const char *fn3_last_error(const fn3_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* FEMNFFT_H */
