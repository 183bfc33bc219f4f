"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

A small driver links the oracle's source directly, built with gcc and the
sanitizers (aborting on the first report), and runs every entry point on
small instances, including the degenerate 1 x 1 and 1 x n shapes, a grid
cost and point clouds.  Any out-of-bounds access, use after free, leak or
undefined arithmetic fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

DRIVER = r"""
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include "pins_oracle.h"

static unsigned long long st = 88172645463325252ULL;
static double unif(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return (double)(st >> 11) / 9007199254740992.0; }

static void marg(double* v, int k) {
    double s = 0.0; int i;
    for (i = 0; i < k; ++i) { v[i] = 0.2 + unif(); s += v[i]; }
    for (i = 0; i < k; ++i) v[i] /= s;
}

static int run(int m, int n, const double* C, double eta, int K) {
    double *a = malloc(sizeof(double) * m), *b = malloc(sizeof(double) * n);
    double *al = malloc(sizeof(double) * m), *be = malloc(sizeof(double) * n);
    double *X = malloc(sizeof(double) * (size_t)m * n), *tr = malloc(sizeof(double) * 8 * (size_t)K);
    oracle_params p; oracle_stats s; int rc, i;
    marg(a, m); marg(b, n);
    oracle_default_params(&p);
    p.eta = eta; p.K = K;
    rc = oracle_pins_trace(m, n, C, a, b, &p, al, be, X, &s, tr);
    if (rc < 0 || !isfinite(s.cost) || !isfinite(s.resid)) { printf("pins %dx%d rc %d\n", m, n, rc); return 1; }
    for (i = 0; i < m; ++i) if (!isfinite(al[i])) return 1;
    rc = oracle_sinkhorn(m, n, C, a, b, eta, 1e-9, 2000, al, be, X, &s);
    if (rc < 0 || !isfinite(s.cost)) { printf("sinkhorn %dx%d rc %d\n", m, n, rc); return 1; }
    printf("%dx%d cost %.6g resid %.3g\n", m, n, s.cost, s.resid);
    free(a); free(b); free(al); free(be); free(X); free(tr);
    return 0;
}

int main(void) {
    int shapes[5][2] = {{1, 1}, {1, 6}, {5, 1}, {7, 5}, {23, 31}};
    int q, k, bad = 0;
    for (q = 0; q < 5; ++q) {
        int m = shapes[q][0], n = shapes[q][1];
        double* C = malloc(sizeof(double) * (size_t)m * n);
        for (k = 0; k < m * n; ++k) C[k] = unif();
        bad |= run(m, n, C, 0.05, 4);
        free(C);
    }
    {
        double* C = malloc(sizeof(double) * 81);
        oracle_cost_grid(3, 0.0, C);
        bad |= run(9, 9, C, 0.05, 5);
        free(C);
    }
    {
        double *x = malloc(sizeof(double) * 6 * 3), *y = malloc(sizeof(double) * 4 * 3);
        double* C = malloc(sizeof(double) * 24);
        for (k = 0; k < 18; ++k) x[k] = unif();
        for (k = 0; k < 12; ++k) y[k] = unif();
        oracle_cost_points(6, 4, 3, x, y, 0.0, C);
        bad |= run(6, 4, C, 0.02, 6);
        free(x); free(y); free(C);
    }
    return bad;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    drv = tmp_path / "drv.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "drv"
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fno-fast-math",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", ORACLE,
           str(drv), os.path.join(ORACLE, "pins_oracle.c"), "-lm", "-o", str(exe)]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.stdout.count("cost") == 7
