/*
 * pins_oracle.h -- FP64 CPU oracle for PINS (arXiv 2502.03749).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, sequential reference
 * against which the HIP path is checked.  Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code
 * with the GPU library.
 *
 * Everything is double precision, sequential index order, libm exp/log.
 * Readings of points the paper leaves open are the same as the GPU path's
 * and are listed in the repository design notes; each function cites the
 * passage it follows.
 */
#ifndef PINS_ORACLE_H
#define PINS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double eta;        /* proximal / entropic parameter (Alg. 2 input) */
    int K;             /* outer EPPA iterations (Alg. 2) */
    int T1;            /* Sinkhorn warm-up cap (Alg. 2) */
    int T2;            /* Newton cap (Alg. 2) */
    double warm_tol;   /* warm-up ends once the row-marginal L1 error <= warm_tol */
    double inner_tol;  /* Newton ends at ||Xe-a||_1+||X^Te-b||_1 <= inner_tol (subproblems 0..K-2) */
    double final_tol;  /* same, last subproblem */
    double cg_rtol;    /* truncated CG: ||res||_2 <= cg_rtol * ||rhs||_2 */
    int cg_max;        /* CG iteration cap */
    double ls_beta;    /* Armijo backtracking factor */
    double ls_c1;      /* Armijo sufficient-increase constant */
    int ls_max;        /* number of trial step sizes 1, beta, beta^2, ... */
    double rho;        /* Sparsify: keep Xt_ij >= rho*10^l*min(a_i,b_j), for the */
    double budget;     /* smallest level l in [0, rho_levels) with nnz <= budget*(m+n-1) */
    int rho_levels;    /* (the densest retained set that fits the budget); no level fitting: nothing kept */
} oracle_params;

typedef struct {
    double cost;       /* <C, X^K> */
    double eps;        /* eta / K */
    double resid;      /* ||X^K e - a||_1 + ||X^K^T e - b||_1 */
    double dual;       /* <a,alpha> + <b,beta> */
    double gap;        /* cost - dual */
    double entropy;    /* -sum X log X */
    int outer, sinkhorn, newton, cg, fallbacks, flags, nnz_last, levels_last;
} oracle_stats;

#define ORACLE_FLAG_LAST_NOT_CONVERGED 1
#define ORACLE_FLAG_INNER_NOT_CONVERGED 2
#define ORACLE_FLAG_NONFINITE 4

void oracle_default_params(oracle_params* p);

/* a0: cost construction (problem statement, eq. (ot)); scale<=0 means 1/max */
int oracle_cost_points(int m, int n, int d, const double* x, const double* y, double scale, double* C);
int oracle_cost_grid(int s, double scale, double* C);

/* Alg. 2 (PINS) on a dense cost.  Outputs: standard-form potentials alpha (m),
 * beta (n) with X^K_ij = exp((alpha_i+beta_j-C_ij)/(eta/K)) and gauge
 * <a,alpha> = <b,beta>; the plan X (m*n row-major, may be NULL). */
int oracle_pins(int m, int n, const double* C, const double* a, const double* b,
                const oracle_params* p, double* alpha, double* beta, double* X, oracle_stats* st);

/* Same, also recording per outer iteration k (8 doubles each, may be NULL):
 * Sinkhorn sweeps, Newton steps, CG iterations, terminal marginal residual,
 * Sparsify level of the last Newton step, <C, X^{k+1}>, nnz(S) of the last
 * Newton step, line-search fallbacks. */
int oracle_pins_trace(int m, int n, const double* C, const double* a, const double* b,
                      const oracle_params* p, double* alpha, double* beta, double* X, oracle_stats* st,
                      double* trace);

/* Alg. 1 (log-domain Sinkhorn) at regularisation eps on C, run until the
 * row-marginal L1 error <= tol or maxit sweeps; standard-form outputs. */
int oracle_sinkhorn(int m, int n, const double* C, const double* a, const double* b,
                    double eps, double tol, int maxit,
                    double* alpha, double* beta, double* X, oracle_stats* st);

/* single steps on an explicit shifted cost Ck, paper-form duals (f, g) */
void oracle_sinkhorn_row(int m, int n, const double* Ck, const double* a, double eta,
                         double* f, const double* g, double* err);
void oracle_sinkhorn_col(int m, int n, const double* Ck, const double* b, double eta,
                         const double* f, double* g);
void oracle_recover(int m, int n, const double* Ck, double eta, const double* f, const double* g,
                    double* X);

#ifdef __cplusplus
}
#endif
#endif
