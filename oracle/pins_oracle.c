/*
 * pins_oracle.c -- FP64 CPU oracle for PINS (arXiv 2502.03749).
 *
 * TEST INFRASTRUCTURE ONLY (see pins_oracle.h).  Plain sequential loops,
 * double precision, libm exp/log/expm1, no blocking, no fusion, no
 * reordering beyond what the algorithm states.
 *
 * Notation follows the paper: C cost, a/b marginals, eta, X^k outer iterate,
 * C^k = C - eta*log X^k shifted cost (Alg. 2), (f, g) inner duals,
 * Xt = recovery map (eq. eppa_x), P^k dual objective (eq. eppa-sub-dual).
 *
 * The outer iterate is kept as the log-plan L^k = log X^k, so the shift
 * C^k = C - eta*L^k never forms log(exp(.)) (which underflows for small eta).
 */
#include "pins_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

void oracle_default_params(oracle_params* p)
{
    /* Hyper-parameters of the numerical appendix (Section "Implementation
     * Details"): T1 = 100, T2 = 50, K = 250, beta = 0.5, c1 = 1e-4, CG
     * relative residual 1e-6, marginal tolerance 1e-9. */
    p->eta = 1e-2;
    p->K = 250;
    p->T1 = 100;
    p->T2 = 50;
    p->warm_tol = 1e-3;
    p->inner_tol = 1e-9;
    p->final_tol = 1e-12;
    p->cg_rtol = 1e-6;
    p->cg_max = 1000;
    p->ls_beta = 0.5;
    p->ls_c1 = 1e-4;
    p->ls_max = 30;
    p->rho = 1e-7;
    p->budget = 64.0;
    p->rho_levels = 11;
}

/* ------------------------------------------------------------------------ */
/* a0: cost                                                                  */
/* ------------------------------------------------------------------------ */

static void scale_cost(long mn, double scale, double* C)
{
    long k;
    if (scale <= 0.0) {
        double mx = 0.0;
        for (k = 0; k < mn; ++k)
            if (C[k] > mx) mx = C[k];
        scale = (mx > 0.0) ? 1.0 / mx : 1.0;
    }
    for (k = 0; k < mn; ++k) C[k] *= scale;
}

int oracle_cost_points(int m, int n, int d, const double* x, const double* y, double scale, double* C)
{
    int i, j, k;
    for (i = 0; i < m; ++i)
        for (j = 0; j < n; ++j) {
            double s = 0.0;
            for (k = 0; k < d; ++k) {
                double t = x[(long)i * d + k] - y[(long)j * d + k];
                s += t * t;
            }
            C[(long)i * n + j] = s;
        }
    scale_cost((long)m * n, scale, C);
    return 0;
}

int oracle_cost_grid(int s, double scale, double* C)
{
    int N = s * s, i, j;
    for (i = 0; i < N; ++i)
        for (j = 0; j < N; ++j) {
            double dr = (double)(i / s - j / s), dc = (double)(i % s - j % s);
            C[(long)i * N + j] = dr * dr + dc * dc;
        }
    if (scale <= 0.0) scale = (s > 1) ? 1.0 / (2.0 * (s - 1) * (s - 1)) : 1.0;
    scale_cost((long)N * N, scale, C);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* primitives                                                               */
/* ------------------------------------------------------------------------ */

/* log(sum_k exp(z_k)) = max z + log sum exp(z - max z) */
static double lse(const double* z, int len)
{
    double mx = -INFINITY, s = 0.0;
    int k;
    for (k = 0; k < len; ++k)
        if (z[k] > mx) mx = z[k];
    if (mx == -INFINITY) return -INFINITY;
    for (k = 0; k < len; ++k) s += exp(z[k] - mx);
    return mx + log(s);
}

/* Alg. 2 f-update: f <- f + eta*(log a - log(Xt(f,g) e)), with
 * log(Xt e)_i = LSE_j((f_i+g_j-Ck_ij-eta)/eta)  (eq. eppa_x).
 * err (optional) receives ||Xt(f_old,g) e - a||_1. */
void oracle_sinkhorn_row(int m, int n, const double* Ck, const double* a, double eta,
                         double* f, const double* g, double* err)
{
    double* z = (double*)malloc(sizeof(double) * (size_t)n);
    double e = 0.0;
    int i, j;
    for (i = 0; i < m; ++i) {
        double l;
        for (j = 0; j < n; ++j) z[j] = (f[i] + g[j] - Ck[(long)i * n + j] - eta) / eta;
        l = lse(z, n);
        e += fabs(exp(l) - a[i]);
        f[i] = f[i] + eta * (log(a[i]) - l);
    }
    if (err) *err = e;
    free(z);
}

/* Alg. 2 g-update with the new f: g <- g + eta*(log b - log(Xt(f,g)^T e)). */
void oracle_sinkhorn_col(int m, int n, const double* Ck, const double* b, double eta,
                         const double* f, double* g)
{
    double* z = (double*)malloc(sizeof(double) * (size_t)m);
    int i, j;
    for (j = 0; j < n; ++j) {
        for (i = 0; i < m; ++i) z[i] = (f[i] + g[j] - Ck[(long)i * n + j] - eta) / eta;
        g[j] = g[j] + eta * (log(b[j]) - lse(z, m));
    }
    free(z);
}

/* recovery map, eq. (eppa_x): Xt = exp((f e^T + e g^T - Ck - eta E)/eta) */
void oracle_recover(int m, int n, const double* Ck, double eta, const double* f, const double* g,
                    double* X)
{
    int i, j;
    for (i = 0; i < m; ++i)
        for (j = 0; j < n; ++j)
            X[(long)i * n + j] = exp((f[i] + g[j] - Ck[(long)i * n + j] - eta) / eta);
}

/* sparsified dual Hessian (up to the factor -1/eta), eq. (eppa-hess):
 * M = [diag(r) S; S^T diag(c)], S stored row-wise (CSR). */
typedef struct {
    int m, n;
    const double *r, *c;
    const int* rp;
    const int* ci;
    const double* v;
} hess_t;

static void hess_apply(const hess_t* H, const double* u, double* y)
{
    int i, j, k;
    for (i = 0; i < H->m; ++i) y[i] = H->r[i] * u[i];
    for (j = 0; j < H->n; ++j) y[H->m + j] = H->c[j] * u[H->m + j];
    for (i = 0; i < H->m; ++i)
        for (k = H->rp[i]; k < H->rp[i + 1]; ++k) {
            j = H->ci[k];
            y[i] += H->v[k] * u[H->m + j];
            y[H->m + j] += H->v[k] * u[i];
        }
}

static double dot(const double* x, const double* y, int len)
{
    double s = 0.0;
    int k;
    for (k = 0; k < len; ++k) s += x[k] * y[k];
    return s;
}

/* truncated CG with Jacobi preconditioner diag(r, c), x0 = 0 (Alg. 2 "CG",
 * Implementation details: relative residual cg_rtol).  Returns iterations. */
static int pcg(const hess_t* H, const double* rhs, double* x, double rtol, int maxit)
{
    int N = H->m + H->n, it, k;
    double *res = (double*)malloc(sizeof(double) * N), *z = (double*)malloc(sizeof(double) * N);
    double *p = (double*)malloc(sizeof(double) * N), *Ap = (double*)malloc(sizeof(double) * N);
    double bnorm = sqrt(dot(rhs, rhs, N)), rz;
    for (k = 0; k < N; ++k) {
        double dg = (k < H->m) ? H->r[k] : H->c[k - H->m];
        x[k] = 0.0;
        res[k] = rhs[k];
        z[k] = res[k] / dg;
        p[k] = z[k];
    }
    rz = dot(res, z, N);
    it = 0;
    if (bnorm > 0.0) {
        while (it < maxit) {
            double pAp, al, be, rz2;
            hess_apply(H, p, Ap);
            pAp = dot(p, Ap, N);
            if (!(pAp > 0.0)) break;
            al = rz / pAp;
            for (k = 0; k < N; ++k) {
                x[k] += al * p[k];
                res[k] -= al * Ap[k];
            }
            ++it;
            if (sqrt(dot(res, res, N)) <= rtol * bnorm) break;
            for (k = 0; k < N; ++k) {
                double dg = (k < H->m) ? H->r[k] : H->c[k - H->m];
                z[k] = res[k] / dg;
            }
            rz2 = dot(res, z, N);
            be = rz2 / rz;
            rz = rz2;
            for (k = 0; k < N; ++k) p[k] = z[k] + be * p[k];
        }
    }
    free(res);
    free(z);
    free(p);
    free(Ap);
    return it;
}

/* ------------------------------------------------------------------------ */
/* Alg. 2                                                                   */
/* ------------------------------------------------------------------------ */

int oracle_pins(int m, int n, const double* C, const double* a, const double* b,
                const oracle_params* p, double* alpha, double* beta, double* X, oracle_stats* st)
{
    return oracle_pins_trace(m, n, C, a, b, p, alpha, beta, X, st, NULL);
}

int oracle_pins_trace(int m, int n, const double* C, const double* a, const double* b,
                      const oracle_params* p, double* alpha, double* beta, double* X, oracle_stats* st,
                      double* trace)
{
    const double eta = p->eta;
    const long mn = (long)m * n;
    int N = m + n, k, t, i, j, l;
    double *L, *Ck, *Xt, *f, *g, *U, *V, *r, *c, *rhs, *d, *loga, *logb;
    int *rp, *ci;
    double* sv;
    long cap = mn;
    oracle_stats S;

    if (m < 1 || n < 1 || !(eta > 0.0) || p->K < 1) return -1;
    memset(&S, 0, sizeof(S));

    L = (double*)malloc(sizeof(double) * mn);
    Ck = (double*)malloc(sizeof(double) * mn);
    Xt = (double*)malloc(sizeof(double) * mn);
    sv = (double*)malloc(sizeof(double) * cap);
    ci = (int*)malloc(sizeof(int) * cap);
    rp = (int*)malloc(sizeof(int) * (m + 1));
    f = (double*)calloc(m, sizeof(double));
    g = (double*)calloc(n, sizeof(double));
    U = (double*)calloc(m, sizeof(double));
    V = (double*)calloc(n, sizeof(double));
    r = (double*)malloc(sizeof(double) * m);
    c = (double*)malloc(sizeof(double) * n);
    rhs = (double*)malloc(sizeof(double) * N);
    d = (double*)malloc(sizeof(double) * N);
    loga = (double*)malloc(sizeof(double) * m);
    logb = (double*)malloc(sizeof(double) * n);
    for (i = 0; i < m; ++i) loga[i] = log(a[i]);
    for (j = 0; j < n; ++j) logb[j] = log(b[j]);

    /* X^0 = a b^T (positive, separable), kept as log X^0; f = g = 0 at k = 0. */
    for (i = 0; i < m; ++i)
        for (j = 0; j < n; ++j) L[(long)i * n + j] = loga[i] + logb[j];

    for (k = 0; k < p->K; ++k) {
        const double tol = (k == p->K - 1) ? p->final_tol : p->inner_tol;
        int converged = 0;
        int sk0 = S.sinkhorn, nt0 = S.newton, cg0 = S.cg, fb0 = S.fallbacks;
        double res_end = 0.0;

        /* shifted cost C^k = C - eta log X^k (Alg. 2) */
        for (long q = 0; q < mn; ++q) Ck[q] = C[q] - eta * L[q];

        /* Sinkhorn warm-up: f-update then g-update (Gauss-Seidel); the row
         * error of the state before each f-update decides the switch. */
        for (t = 0; t < p->T1; ++t) {
            double err;
            oracle_sinkhorn_row(m, n, Ck, a, eta, f, g, &err);
            oracle_sinkhorn_col(m, n, Ck, b, eta, f, g);
            S.sinkhorn++;
            if (err <= p->warm_tol) break;
        }

        /* sparse Newton refinement */
        for (t = 0;; ++t) {
            double res = 0.0, gd, fa, ub, da, db;
            long nnz;
            int lev, cgit, accepted = 0, h;
            hess_t H;

            oracle_recover(m, n, Ck, eta, f, g, Xt);
            for (i = 0; i < m; ++i) r[i] = 0.0;
            for (j = 0; j < n; ++j) c[j] = 0.0;
            for (i = 0; i < m; ++i)
                for (j = 0; j < n; ++j) {
                    r[i] += Xt[(long)i * n + j];
                    c[j] += Xt[(long)i * n + j];
                }
            for (i = 0; i < m; ++i) res += fabs(a[i] - r[i]);
            for (j = 0; j < n; ++j) res += fabs(b[j] - c[j]);
            res_end = res;
            if (!isfinite(res)) {
                S.flags |= ORACLE_FLAG_NONFINITE;
                break;
            }
            if (res <= tol) {
                converged = 1;
                break;
            }
            if (t == p->T2) break;

            /* Sparsify(Hessian, rho): first threshold level whose kept count fits
             * the budget; when none does, no entry is kept (lev = rho_levels,
             * threshold +inf) and the Newton system is its diagonal */
            lev = p->rho_levels;
            for (l = 0; l < p->rho_levels; ++l) {
                double rl = p->rho * pow(10.0, (double)l);
                nnz = 0;
                for (i = 0; i < m; ++i)
                    for (j = 0; j < n; ++j) {
                        double mn_ab = a[i] < b[j] ? a[i] : b[j];
                        if (Xt[(long)i * n + j] >= rl * mn_ab) ++nnz;
                    }
                if ((double)nnz <= p->budget * (double)(m + n - 1)) {
                    lev = l;
                    break;
                }
            }
            {
                double rl = (lev < p->rho_levels) ? p->rho * pow(10.0, (double)lev) : INFINITY;
                nnz = 0;
                rp[0] = 0;
                for (i = 0; i < m; ++i) {
                    for (j = 0; j < n; ++j) {
                        double mn_ab = a[i] < b[j] ? a[i] : b[j];
                        if (Xt[(long)i * n + j] >= rl * mn_ab) {
                            ci[nnz] = j;
                            sv[nnz] = Xt[(long)i * n + j];
                            ++nnz;
                        }
                    }
                    rp[i + 1] = (int)nnz;
                }
            }
            S.nnz_last = (int)nnz;
            S.levels_last = lev;

            /* CG on M d = eta * grad P,  M = -eta * Hessian (eq. eppa-hess) */
            for (i = 0; i < m; ++i) rhs[i] = eta * (a[i] - r[i]);
            for (j = 0; j < n; ++j) rhs[m + j] = eta * (b[j] - c[j]);
            H.m = m; H.n = n; H.r = r; H.c = c; H.rp = rp; H.ci = ci; H.v = sv;
            cgit = pcg(&H, rhs, d, p->cg_rtol, p->cg_max);
            S.cg += cgit;

            /* Armijo backtracking on P^k (eq. eppa-sub-dual):
             *   P(f+al df, g+al dg) - P(f,g)
             *     = al(<a,df>+<b,dg>) - eta*sum_ij Xt_ij*expm1(al(df_i+dg_j)/eta)
             * accept the first al = beta^h with increase >= c1*al*<grad P, d>. */
            gd = 0.0;
            da = 0.0;
            db = 0.0;
            fa = 0.0;
            for (i = 0; i < m; ++i) {
                gd += (a[i] - r[i]) * d[i];
                da += a[i] * d[i];
                fa += fabs(a[i] * d[i]);
            }
            for (j = 0; j < n; ++j) {
                gd += (b[j] - c[j]) * d[m + j];
                db += b[j] * d[m + j];
                fa += fabs(b[j] * d[m + j]);
            }
            ub = 64.0 * DBL_EPSILON * fa; /* resolution of the increase evaluation */
            if (gd > 0.0 && p->ls_c1 * gd <= ub) {
                accepted = 1;
                ub = 1.0;
            } else if (gd > 0.0) {
                double al = 1.0;
                for (h = 0; h < p->ls_max; ++h, al *= p->ls_beta) {
                    double sm = 0.0, inc;
                    for (i = 0; i < m; ++i)
                        for (j = 0; j < n; ++j)
                            sm += Xt[(long)i * n + j] * expm1(al * (d[i] + d[m + j]) / eta);
                    inc = al * (da + db) - eta * sm;
                    if (inc >= p->ls_c1 * al * gd) {
                        accepted = 1;
                        ub = al;
                        break;
                    }
                }
            }
            if (accepted) {
                for (i = 0; i < m; ++i) f[i] += ub * d[i];
                for (j = 0; j < n; ++j) g[j] += ub * d[m + j];
            } else {
                /* no ascent step found: one Sinkhorn iteration (monotone ascent) instead */
                oracle_sinkhorn_row(m, n, Ck, a, eta, f, g, NULL);
                oracle_sinkhorn_col(m, n, Ck, b, eta, f, g);
                S.fallbacks++;
            }
            S.newton++;
        }
        if (!converged) S.flags |= (k == p->K - 1) ? ORACLE_FLAG_LAST_NOT_CONVERGED : ORACLE_FLAG_INNER_NOT_CONVERGED;

        /* X^{k+1} = Xt^k(f, g), kept as its log (eq. eppa_x) */
        for (i = 0; i < m; ++i)
            for (j = 0; j < n; ++j) {
                long q = (long)i * n + j;
                L[q] = (f[i] + g[j] - Ck[q] - eta) / eta;
            }
        for (i = 0; i < m; ++i) U[i] += f[i];
        for (j = 0; j < n; ++j) V[j] += g[j];
        S.outer++;
        if (trace) {
            double cst = 0.0;
            for (long q = 0; q < mn; ++q) cst += C[q] * exp(L[q]);
            trace[8 * k + 0] = S.sinkhorn - sk0;
            trace[8 * k + 1] = S.newton - nt0;
            trace[8 * k + 2] = S.cg - cg0;
            trace[8 * k + 3] = res_end;
            trace[8 * k + 4] = S.levels_last;
            trace[8 * k + 5] = cst;
            trace[8 * k + 6] = (S.newton > nt0) ? S.nnz_last : 0;
            trace[8 * k + 7] = S.fallbacks - fb0;
        }
    }

    /* Output X^K, and standard-form potentials at eps = eta/K:
     * alpha = (U + eta log a)/K - eta, beta = (V + eta log b)/K, where U, V
     * are the sums of the terminal inner duals; gauge <a,alpha> = <b,beta>. */
    {
        const double K = (double)p->K, eps = eta / K;
        double sa = 0.0, sb = 0.0, tg, cost = 0.0, ent = 0.0, res = 0.0;
        for (i = 0; i < m; ++i) alpha[i] = (U[i] + eta * loga[i]) / K - eta;
        for (j = 0; j < n; ++j) beta[j] = (V[j] + eta * logb[j]) / K;
        for (i = 0; i < m; ++i) sa += a[i] * alpha[i];
        for (j = 0; j < n; ++j) sb += b[j] * beta[j];
        tg = 0.5 * (sb - sa);
        for (i = 0; i < m; ++i) alpha[i] += tg;
        for (j = 0; j < n; ++j) beta[j] -= tg;
        for (i = 0; i < m; ++i) r[i] = 0.0;
        for (j = 0; j < n; ++j) c[j] = 0.0;
        for (i = 0; i < m; ++i)
            for (j = 0; j < n; ++j) {
                long q = (long)i * n + j;
                double x = exp(L[q]);
                if (X) X[q] = x;
                cost += C[q] * x;
                if (x > 0.0) ent -= x * L[q];
                r[i] += x;
                c[j] += x;
            }
        for (i = 0; i < m; ++i) res += fabs(r[i] - a[i]);
        for (j = 0; j < n; ++j) res += fabs(c[j] - b[j]);
        S.cost = cost;
        S.eps = eps;
        S.resid = res;
        S.entropy = ent;
        S.dual = 0.0;
        for (i = 0; i < m; ++i) S.dual += a[i] * alpha[i];
        for (j = 0; j < n; ++j) S.dual += b[j] * beta[j];
        S.gap = cost - S.dual;
        if (!isfinite(cost)) S.flags |= ORACLE_FLAG_NONFINITE;
    }
    if (st) *st = S;

    free(L); free(Ck); free(Xt); free(sv); free(ci); free(rp);
    free(f); free(g); free(U); free(V); free(r); free(c); free(rhs); free(d);
    free(loga); free(logb);
    return (S.flags & ORACLE_FLAG_NONFINITE) ? -4 : ((S.flags & ORACLE_FLAG_LAST_NOT_CONVERGED) ? 1 : 0);
}

/* ------------------------------------------------------------------------ */
/* Alg. 1, plain log-domain Sinkhorn at regularisation eps                  */
/* ------------------------------------------------------------------------ */

int oracle_sinkhorn(int m, int n, const double* C, const double* a, const double* b,
                    double eps, double tol, int maxit,
                    double* alpha, double* beta, double* X, oracle_stats* st)
{
    double *f = (double*)calloc(m, sizeof(double)), *g = (double*)calloc(n, sizeof(double));
    double* Xw = (double*)malloc(sizeof(double) * (long)m * n);
    double err = INFINITY;
    int it, i, j, conv = 0;
    oracle_stats S;
    memset(&S, 0, sizeof(S));
    for (it = 0; it < maxit; ++it) {
        oracle_sinkhorn_row(m, n, C, a, eps, f, g, &err);
        if (err <= tol && it > 0) { /* state before this f-update already met tol */
            conv = 1;
            break;
        }
        oracle_sinkhorn_col(m, n, C, b, eps, f, g);
        S.sinkhorn++;
    }
    if (!conv) {
        /* finish with a g-update so that the column marginals are exact */
    } else {
        oracle_sinkhorn_col(m, n, C, b, eps, f, g);
    }
    {
        double sa = 0.0, sb = 0.0, tg, res = 0.0, cost = 0.0, ent = 0.0;
        double *r = (double*)calloc(m, sizeof(double)), *c = (double*)calloc(n, sizeof(double));
        for (i = 0; i < m; ++i) alpha[i] = f[i] - eps; /* X = exp((f+g-C-eps)/eps) */
        for (j = 0; j < n; ++j) beta[j] = g[j];
        for (i = 0; i < m; ++i) sa += a[i] * alpha[i];
        for (j = 0; j < n; ++j) sb += b[j] * beta[j];
        tg = 0.5 * (sb - sa);
        for (i = 0; i < m; ++i) alpha[i] += tg;
        for (j = 0; j < n; ++j) beta[j] -= tg;
        for (i = 0; i < m; ++i)
            for (j = 0; j < n; ++j) {
                long q = (long)i * n + j;
                double lx = (alpha[i] + beta[j] - C[q]) / eps, x = exp(lx);
                Xw[q] = x;
                cost += C[q] * x;
                if (x > 0.0) ent -= x * lx;
                r[i] += x;
                c[j] += x;
            }
        for (i = 0; i < m; ++i) res += fabs(r[i] - a[i]);
        for (j = 0; j < n; ++j) res += fabs(c[j] - b[j]);
        if (X) memcpy(X, Xw, sizeof(double) * (long)m * n);
        S.cost = cost;
        S.eps = eps;
        S.resid = res;
        S.entropy = ent;
        for (i = 0; i < m; ++i) S.dual += a[i] * alpha[i];
        for (j = 0; j < n; ++j) S.dual += b[j] * beta[j];
        S.gap = cost - S.dual;
        S.outer = 1;
        S.flags = conv ? 0 : ORACLE_FLAG_LAST_NOT_CONVERGED;
        free(r);
        free(c);
    }
    if (st) *st = S;
    free(f);
    free(g);
    free(Xw);
    return conv ? 0 : 1;
}
