/*
 * Oracle O1 -- TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the
 * bench's CPU-baseline leg may load this library; the product path never does.
 *
 * Plain FP64 direct O(N_t * N_s) evaluation of the discrete Green sum that the
 * fast method approximates:
 *
 *   phi(r_i) = sum_j q_j w_j G(r_i - r_j),   G(r) = -(1/2pi) ln|r|
 *       (the paper's eq. (2), with the volume and surface terms merged into one
 *        list of quadrature points r_j of weight w_j = omega_j det J(r_j);
 *        G is the 2D Green function given with eq. (1))
 *   H(r_i)   = -grad phi(r_i) = (1/2pi) sum_j q_j w_j (r_i - r_j)/|r_i - r_j|^2
 *       (the field/potential relation H = -grad phi stated in the introduction)
 *
 * and the exact transposes of both maps with respect to the charges q:
 *
 *   u_j = w_j sum_i v_i G(r_i - r_j)                              (phi^T)
 *   u_j = w_j sum_i V_i . (1/2pi)(r_i - r_j)/|r_i - r_j|^2        (H^T)
 *
 * Pairs at distance exactly zero are skipped (the singular self term of a
 * point source is not part of the sum).  Every sum over the long index is
 * Neumaier-compensated, so the result is accurate to a few ulps of the sum of
 * magnitudes.  No FFT, no binning, no cut-off.  Parity unpinned: none (pinned
 * by the closed forms and invariants in tests/test_oracle_*.py).
 *
 * Arrays of 2-vectors are interleaved [n][2] (x, y), row-major, FP64.
 * OpenMP parallel over the output index; each output is summed serially in
 * index order, so results do not depend on the thread count.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#define INV_2PI 0.15915494309189533576888376337251436

typedef struct { double s, c; } acc_t;

static inline void acc_add(acc_t *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static inline double acc_val(const acc_t *a) { return a->s + a->c; }

int o1_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* phi[nt] and/or H[nt][2] at targets y[nt][2] from sources x[ns][2] with
 * weights w[ns] and charges q[ns].  Either output may be NULL. */
int o1_forward(int64_t nt, const double *y, int64_t ns, const double *x,
               const double *w, const double *q, double *phi, double *H)
{
    if (nt < 0 || ns < 0 || !y || !x || !w || !q) return 1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < nt; ++i) {
        const double yx = y[2 * i], yy = y[2 * i + 1];
        acc_t ap = {0, 0}, ahx = {0, 0}, ahy = {0, 0};
        for (int64_t j = 0; j < ns; ++j) {
            const double dx = yx - x[2 * j], dy = yy - x[2 * j + 1];
            const double r2 = dx * dx + dy * dy;
            if (r2 == 0.0) continue;
            const double s = w[j] * q[j];
            if (phi) acc_add(&ap, -0.5 * INV_2PI * s * log(r2));
            if (H) {
                const double f = INV_2PI * s / r2;
                acc_add(&ahx, f * dx);
                acc_add(&ahy, f * dy);
            }
        }
        if (phi) phi[i] = acc_val(&ap);
        if (H) { H[2 * i] = acc_val(&ahx); H[2 * i + 1] = acc_val(&ahy); }
    }
    return 0;
}

/* u[ns] = w_j * sum_i ( v_i G(y_i - x_j) + V_i . (1/2pi)(y_i - x_j)/|y_i - x_j|^2 ).
 * v (nt) and/or V (nt x 2) may be NULL (that term is then absent). */
int o1_adjoint(int64_t nt, const double *y, int64_t ns, const double *x,
               const double *w, const double *v, const double *V, double *u)
{
    if (nt < 0 || ns < 0 || !y || !x || !w || !u) return 1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < ns; ++j) {
        const double xx = x[2 * j], xy = x[2 * j + 1];
        acc_t a = {0, 0};
        for (int64_t i = 0; i < nt; ++i) {
            const double dx = y[2 * i] - xx, dy = y[2 * i + 1] - xy;
            const double r2 = dx * dx + dy * dy;
            if (r2 == 0.0) continue;
            if (v) acc_add(&a, -0.5 * INV_2PI * v[i] * log(r2));
            if (V) acc_add(&a, INV_2PI * (V[2 * i] * dx + V[2 * i + 1] * dy) / r2);
        }
        u[j] = w[j] * acc_val(&a);
    }
    return 0;
}
