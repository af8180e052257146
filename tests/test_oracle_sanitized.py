"""The direct-sum oracles (oracle/direct.c, oracle/direct3.c) built with AddressSanitizer and
UndefinedBehaviorSanitizer on the host and driven through every entry point -- empty sets,
NULL outputs, coincident points, ragged sizes -- must run clean (any report aborts the run) and
print the same results as a plain build of the same driver.  CPU only."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
int o1_forward(int64_t, const double *, int64_t, const double *, const double *, const double *, double *, double *);
int o1_adjoint(int64_t, const double *, int64_t, const double *, const double *, const double *, const double *,
               double *);
int o1_3d_forward(int64_t, const double *, int64_t, const double *, const double *, const double *, double *,
                  double *);
int o1_3d_adjoint(int64_t, const double *, int64_t, const double *, const double *, const double *, const double *,
                  double *);

static uint64_t st = 88172645463325252ull;
static double rnd(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return (st >> 11) * (1.0 / 9007199254740992.0); }
static double *arr(int64_t n) { double *p = malloc(sizeof(double) * (n > 0 ? n : 1)); for (int64_t i = 0; i < n; ++i) p[i] = rnd() - 0.5; return p; }
static double sum(const double *p, int64_t n) { double s = 0; for (int64_t i = 0; i < n; ++i) s += p[i] * (1.0 + 1e-3 * i); return s; }

int main(void)
{
    const int64_t sizes[][2] = {{0, 0}, {0, 5}, {5, 0}, {1, 1}, {7, 13}, {64, 33}, {200, 301}};
    for (unsigned c = 0; c < sizeof sizes / sizeof sizes[0]; ++c) {
        const int64_t nt = sizes[c][0], ns = sizes[c][1];
        for (int dim = 2; dim <= 3; ++dim) {
            double *y = arr(dim * nt), *x = arr(dim * ns), *w = arr(ns), *q = arr(ns), *v = arr(nt), *V = arr(dim * nt);
            for (int64_t j = 0; j < ns; ++j) w[j] += 1.0;
            if (nt > 2 && ns > 2) for (int d = 0; d < dim; ++d) y[d] = x[dim + d];  /* a coincident pair */
            double *phi = arr(nt), *H = arr(dim * nt), *u = arr(ns);
            int rc;
            if (dim == 2) {
                rc = o1_forward(nt, y, ns, x, w, q, phi, H) | o1_forward(nt, y, ns, x, w, q, NULL, H) |
                     o1_forward(nt, y, ns, x, w, q, phi, NULL);
                printf("2d %lld %lld fwd %d %.17g %.17g\n", (long long)nt, (long long)ns, rc, sum(phi, nt), sum(H, 2 * nt));
                rc = o1_adjoint(nt, y, ns, x, w, v, V, u);
                printf("2d adj %d %.17g\n", rc, sum(u, ns));
                rc = o1_adjoint(nt, y, ns, x, w, NULL, V, u);
                printf("2d adjH %d %.17g\n", rc, sum(u, ns));
            } else {
                rc = o1_3d_forward(nt, y, ns, x, w, q, phi, H) | o1_3d_forward(nt, y, ns, x, w, q, NULL, H);
                printf("3d %lld %lld fwd %d %.17g %.17g\n", (long long)nt, (long long)ns, rc, sum(phi, nt), sum(H, 3 * nt));
                rc = o1_3d_adjoint(nt, y, ns, x, w, v, V, u);
                printf("3d adj %d %.17g\n", rc, sum(u, ns));
            }
            printf("null args %d %d\n", o1_forward(-1, y, ns, x, w, q, phi, H), o1_3d_adjoint(nt, NULL, ns, x, w, v, V, u));
            free(y); free(x); free(w); free(q); free(v); free(V); free(phi); free(H); free(u);
        }
    }
    return 0;
}
"""


def _build(tmp, name, extra):
    drv = os.path.join(tmp, "driver.c")
    with open(drv, "w") as f:
        f.write(DRIVER)
    exe = os.path.join(tmp, name)
    cmd = ["gcc", "-O1", "-g", "-ffp-contract=off", *extra, drv, os.path.join(ORACLE, "direct.c"),
           os.path.join(ORACLE, "direct3.c"), "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_direct_sum_oracles_run_clean_under_asan_and_ubsan(tmp_path):
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    plain = _build(str(tmp_path), "plain", [])
    checked = _build(str(tmp_path), "checked", san)
    # verify_asan_link_order=0: other preloaded libraries of the environment may come first
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    a = subprocess.run([plain], capture_output=True, text=True, timeout=300)
    b = subprocess.run([checked], capture_output=True, text=True, timeout=300, env=env)
    assert a.returncode == 0 and b.returncode == 0, b.stderr[-2000:]
    assert "runtime error" not in b.stderr and "ERROR: AddressSanitizer" not in b.stderr, b.stderr[-2000:]
    assert a.stdout == b.stdout and a.stdout.count("\n") > 40
