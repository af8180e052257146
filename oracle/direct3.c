/*
 * Oracle O1 in 3D -- TEST INFRASTRUCTURE ONLY.  Only tests/ and the smoke check may
 * load this library; the product path never does.
 *
 * Plain FP64 direct O(N_t * N_s) evaluation of the discrete Green sum of the paper's
 * eq. (2) with the 3D Green function given with eq. (1), G(r) = 1/(4 pi |r|):
 *
 *   phi(r_i) = sum_j q_j w_j / (4 pi |r_i - r_j|)
 *   H(r_i)   = -grad phi(r_i) = (1/4pi) sum_j q_j w_j (r_i - r_j) / |r_i - r_j|^3
 *
 * and the exact transposes of both maps with respect to the charges q:
 *
 *   u_j = w_j sum_i v_i / (4 pi |r_i - r_j|)                              (phi^T)
 *   u_j = w_j sum_i V_i . (1/4pi) (r_i - r_j) / |r_i - r_j|^3             (H^T)
 *
 * Pairs at distance exactly zero are skipped.  Neumaier-compensated sums over the long
 * index; OpenMP over the output index, each output summed serially in index order.
 * 3-vectors are interleaved [n][3], FP64.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#define INV_4PI 0.07957747154594766788444188168625718

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

/* phi[nt] and/or H[nt][3] at targets y[nt][3] from sources x[ns][3], weights w, charges q. */
int o1_3d_forward(int64_t nt, const double *y, int64_t ns, const double *x,
                  const double *w, const double *q, double *phi, double *H)
{
    if (nt < 0 || ns < 0 || !y || !x || !w || !q) return 1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < nt; ++i) {
        const double y0 = y[3 * i], y1 = y[3 * i + 1], y2 = y[3 * i + 2];
        acc_t ap = {0, 0}, a0 = {0, 0}, a1 = {0, 0}, a2 = {0, 0};
        for (int64_t j = 0; j < ns; ++j) {
            const double d0 = y0 - x[3 * j], d1 = y1 - x[3 * j + 1], d2 = y2 - x[3 * j + 2];
            const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
            if (r2 == 0.0) continue;
            const double r = sqrt(r2);
            const double s = INV_4PI * w[j] * q[j];
            if (phi) acc_add(&ap, s / r);
            if (H) {
                const double f = s / (r2 * r);
                acc_add(&a0, f * d0);
                acc_add(&a1, f * d1);
                acc_add(&a2, f * d2);
            }
        }
        if (phi) phi[i] = acc_val(&ap);
        if (H) {
            H[3 * i] = acc_val(&a0);
            H[3 * i + 1] = acc_val(&a1);
            H[3 * i + 2] = acc_val(&a2);
        }
    }
    return 0;
}

/* u[ns] = w_j sum_i ( v_i G(y_i - x_j) + V_i . (1/4pi)(y_i - x_j)/|y_i - x_j|^3 ); v or V may be NULL. */
int o1_3d_adjoint(int64_t nt, const double *y, int64_t ns, const double *x,
                  const double *w, const double *v, const double *V, double *u)
{
    if (nt < 0 || ns < 0 || !y || !x || !w || !u) return 1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < ns; ++j) {
        const double x0 = x[3 * j], x1 = x[3 * j + 1], x2 = x[3 * j + 2];
        acc_t a = {0, 0};
        for (int64_t i = 0; i < nt; ++i) {
            const double d0 = y[3 * i] - x0, d1 = y[3 * i + 1] - x1, d2 = y[3 * i + 2] - x2;
            const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
            if (r2 == 0.0) continue;
            const double r = sqrt(r2);
            if (v) acc_add(&a, INV_4PI * v[i] / r);
            if (V) acc_add(&a, INV_4PI * (V[3 * i] * d0 + V[3 * i + 1] * d1 + V[3 * i + 2] * d2) / (r2 * r));
        }
        u[j] = w[j] * acc_val(&a);
    }
    return 0;
}
