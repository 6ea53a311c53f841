/*
 * FP64 CPU oracle for entropy-regularized optimal transport (EOT) solved by
 * log-domain Sinkhorn and by Acc-Sinkhorn with homotopy.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plainly written reference
 * that the GPU library is checked against.  It shares no code, header, table
 * or helper with the HIP library; the library never calls it.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * Everything is double precision.  Loops are written in the order of the
 * paper's definitions; OpenMP only splits independent rows (or independent
 * columns) between threads, never a single sum.
 *
 * Notation (paper, Sec. 2 "Dual Formulation"): the cost is divided by eps
 * (Ct = C/eps), so the problem is solved at eps = 1;
 *   P_ij(u,v) = exp(u_i + v_j - Ct_ij)                       eq:P-from-dual
 *   F(u,v)    = sum_ij P_ij - <u,a> - <v,b>                  eq:dual-obj
 *   u(v)_i    = log a_i - LSE_j(v_j - Ct_ij)                 eq:u-update (exact row solve)
 *   f(v)      = F(u(v),v) = 1 - <u(v),a> - <v,b>            Lemma coercivity (App. A)
 *   grad f(v) = c_P(u(v),v) - b                              eq:grad-f
 *   Sinkhorn(v) = v - P_Nperp grad phi*(P_Nperp grad f(v))   eq:normalized-sinkhorn
 * with grad phi*(xi) = log(1 + xi./b) (Sec. 3).  For v with sum(v) = 0 and
 * sum_j c_P,j = 1 this equals center(log b - ell), ell_j = LSE_i(u_i - Ct_ij),
 * which is the form used here (log domain, Sec. 5 "Color Transfer").
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* log(sum_k exp(z_k)) with the max shift of the log-domain method. */
static double lse_strided(const double *z, int64_t count, int64_t stride)
{
    double mx = -INFINITY;
    for (int64_t k = 0; k < count; k++) {
        double t = z[k * stride];
        if (t > mx) mx = t;
    }
    if (mx == -INFINITY) return -INFINITY;
    double s = 0.0;
    for (int64_t k = 0; k < count; k++) s += exp(z[k * stride] - mx);
    return mx + log(s);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/*
 * Exact row solve, eq:u-update: u_i = log a_i - LSE_j(x_j - C_ij/eps).
 * Returns <u,a>.
 */
static double row_solve(const double *C, int64_t n, int64_t m, double eps,
                        const double *a, const double *x, double *u)
{
    double ua = 0.0;
#pragma omp parallel
    {
        double *z = (double *)malloc(sizeof(double) * (size_t)m);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; i++) {
            for (int64_t j = 0; j < m; j++) z[j] = x[j] - C[i * m + j] / eps;
            u[i] = log(a[i]) - lse_strided(z, m, 1);
        }
        free(z);
    }
    for (int64_t i = 0; i < n; i++) ua += u[i] * a[i];
    return ua;
}

/* ell_j = LSE_i(u_i - C_ij/eps): log of the column sums of P without exp(x_j). */
static void col_lse(const double *C, int64_t n, int64_t m, double eps,
                    const double *u, double *ell)
{
#pragma omp parallel
    {
        double *z = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp for schedule(static)
        for (int64_t j = 0; j < m; j++) {
            for (int64_t i = 0; i < n; i++) z[i] = u[i] - C[i * m + j] / eps;
            ell[j] = lse_strided(z, n, 1);
        }
        free(z);
    }
}

/*
 * One normalized Sinkhorn step at x (eq:normalized-sinkhorn, log-domain form).
 * Outputs: u = u(x); ell; S = Sinkhorn(x) = center(log b - ell);
 * err = sum_j |c_j - b_j| with c_j = exp(x_j + ell_j) (the column part of the
 * stopping rule eq:l1tol; the row part is zero by construction of u(x));
 * fval = f(x) = 1 - <u,a> - <x,b>.
 */
void oracle_sstep(const double *C, int64_t n, int64_t m, double eps,
                  const double *a, const double *b, const double *x,
                  double *u, double *ell, double *S, double *err, double *fval)
{
    double ua = row_solve(C, n, m, eps, a, x, u);
    col_lse(C, n, m, eps, u, ell);
    double xb = 0.0, e = 0.0, mean = 0.0;
    for (int64_t j = 0; j < m; j++) {
        xb += x[j] * b[j];
        e += fabs(exp(x[j] + ell[j]) - b[j]);
        S[j] = log(b[j]) - ell[j];
        mean += S[j];
    }
    mean /= (double)m;
    for (int64_t j = 0; j < m; j++) S[j] -= mean;
    *err = e;
    *fval = 1.0 - ua - xb;
}

enum { ORACLE_SINKHORN = 0, ORACLE_ACC = 1 };
enum { ORACLE_W_LITERAL = 0, ORACLE_W_Y_CONTINUOUS = 1 };

/*
 * Full solve.  a, b must already sum to one (eq:Fc requires 1'a = 1'b = 1).
 *
 * method ORACLE_SINKHORN: v_0 = 0, v_{k+1} = Sinkhorn(v_k) (eq:normalized-sinkhorn),
 *   stop as soon as err(v_k) < tol or k = max_iter.
 * method ORACLE_ACC: Algorithm A2MD inside the homotopy of Algorithm
 *   A2MD-homotopy.  x_0 = w_0 = 0; per stage alpha = sqrt(2 mu);
 *     x_{k+1} = (w_k + Sinkhorn(x_k)) / (1 + alpha)
 *     w_{k+1} = (w_k + (alpha^2 - 2) x_{k+1} + 2 Sinkhorn(x_{k+1})) / (1 + alpha)
 *   Sinkhorn(x_{k+1}) is kept for the next x-update (one step per iteration).
 *   After m_stage inner iterations: mu <- mu/2, m_stage <- floor(sqrt(2) m_stage) + 1.
 *   The stopping rule is tested at every new x (inner iteration).
 *   w_rule ORACLE_W_Y_CONTINUOUS rescales w by alpha_new/alpha_old at a stage
 *   change so that y = w/alpha is carried over; ORACLE_W_LITERAL passes w as printed.
 *
 * Outputs: f = eps*u(x), g = eps*x at the returned iterate; iters = It;
 * steps = number of Sinkhorn steps evaluated; err at the returned iterate.
 * Optional traces (length max_iter+1, may be NULL): err and f(x) per It;
 * trace_x (length (max_iter+1)*m, may be NULL): the iterate x per It.
 * Returns 1 if converged (err < tol), 0 otherwise.
 */
/*
 * Stability monitor (not part of the paper's algorithm; a safeguard of this
 * build, off unless `restart` is set).  The reduced dual objective
 * f(x) = 1 - <u(x),a> - <x,b> (Lemma coercivity, App. A) decreases along plain
 * Sinkhorn (Lemma sinkhorn-descent); Acc-Sinkhorn need not decrease it at every
 * step.  After each accepted Acc iterate, f(x_k) > f(x_{k-1}) + delta counts as
 * an increase, delta = 1e-8 + 1e-12 |f(x_k)| (above the rounding of f computed
 * from FP32 exponentials).  With `restart`, an increase also resets the
 * extrapolation variable to the current iterate, w <- alpha x (y = x), the
 * function-value restart of accelerated methods.  Counts go to *n_increase and
 * *n_restart (either may be NULL).
 */
static int stability_increase(double fval, double fprev)
{
    return fval > fprev + (1e-8 + 1e-12 * fabs(fval));
}

/*
 * Boundedness conditions of the Acc iterates (App. B, Theorem
 * thm:condition-boundedness) and the shifted Lyapunov function of its proof,
 * evaluated along the run (a monitor: the solve itself is unchanged).
 *
 * For an iterate (x_k, w_k) with column sums c = c_P(u(x_k), x_k):
 *   grad f(x_k) = xi = c - b                                   eq:grad-f
 *   p = grad phi*(xi) = log(c ./ b)                            Sec. 3
 *   D_k = diag(b (e^p - 1) ./ p) = diag(xi ./ p)               eq:D (the logarithmic mean of c_j and b_j,
 *                                                              b_j at c_j = b_j: series for |p| < 1e-3)
 *   K_k = D_phi*(0, xi) = sum_j (xi_j - b_j p_j) = KL(b || c)  (generalized KL; series for |p| < 1e-3)
 *   v_k = y_k - x_k = w_k / alpha - x_k                        (w = alpha y, Sec. 4)
 *   E_k = f(x_k) + (mu/2) ||v_k||^2_{D_k} - theta/(1+alpha) K_k,  theta = (1/2 + alpha)/(1 + alpha)
 *     (the proof's shifted Lyapunov function with L = 1, without the constant f(x*))
 * and for consecutive iterates (k, k+1) of one homotopy stage:
 *   condition 1:  ||xi_k||^2_{D_k^-1 D_k+1 D_k^-1} < (4 - alpha^2 - 2 alpha^(1/2)) / (2 alpha (1+alpha)^2) K_k
 *   condition 2:  ||v_k||^2_{D_k+1 - D_k} < alpha^(3/2) ||v_k+1||^2_{D_k+1}
 *     (the printed ||v_k||_{D_k+1 - D_k} < alpha^(3/4) ||v_k+1||_{D_k+1}, squared; a negative left side
 *     satisfies it)
 *   Lyapunov rise:  E_k+1 > E_k + 1e-8 + 1e-12 |f(x_k+1)| + 1e-6 ((mu/2) ||v_k+1||^2_D + ||xi_k+1||_1)
 *     (a noise threshold for values computed from FP32 exponentials).
 * Both conditions are checked with the alpha the algorithm runs with (the
 * theorem states them for alpha^2 = mu/L).  The iterate w_k is the value
 * carried to the next x update (after a restart reset).  At a stage change the
 * last iterate, with w as handed to the new stage and the new stage's alpha
 * and mu, is the first iterate of the next stage.
 */
typedef struct {
    int64_t m;
    double *xi, *D, *v;   /* the last iterate's grad f, metric diagonal and v */
    double K, E, fval;    /* its D_phi*(0, grad f), shifted Lyapunov value and f(x) */
    int have;
    int64_t n1, n2, nl;   /* violations of conditions 1 and 2, Lyapunov rises */
} cond_mon;

/* D_jj (eq:D) and the j-term of D_phi*(0, xi) from c_j and b_j:
 * D = b (e^p - 1)/p = b sum_{k>=0} p^k/(k+1)!,  K = b (e^p - 1 - p) = b sum_{k>=2} p^k/k!,
 * summed as series for |p| < 1e-2 (where e^p - 1 - p would cancel), else in closed form. */
static void metric_terms(double c, double b, double *xi, double *D, double *K)
{
    *xi = c - b;
    const double p = log1p(*xi / b);
    if (fabs(p) < 1e-2) {
        double term = 1.0, sd = 0.0, sk = 0.0;  /* term = p^k / (k+1)! */
        for (int k = 0; k <= 8; k++) {
            sd += term;
            if (k >= 1) sk += term * p;          /* p^(k+1)/(k+1)!, k+1 >= 2 */
            term *= p / (double)(k + 2);
        }
        *D = b * sd;
        *K = b * sk;
    } else {
        *D = *xi / p;
        *K = *xi - b * p;
    }
}

static double lyap_theta(double alpha) { return (0.5 + alpha) / (1.0 + alpha); }

/* The monitor's metric for given column sums: D_jj (eq:D) and the terms of
 * D_phi*(0, c - b) (exposed for the tests that pin them). */
void oracle_cond_metric(const double *c, const double *b, int64_t m, double *D, double *K)
{
    for (int64_t j = 0; j < m; j++) {
        double xi;
        metric_terms(c[j], b[j], &xi, &D[j], &K[j]);
    }
}

/* The Lyapunov value of the stored iterate under (alpha, mu); v recomputed from w, x. */
static double mon_rebase(cond_mon *M, const double *x, const double *w, double alpha, double mu)
{
    double vd = 0.0;
    for (int64_t j = 0; j < M->m; j++) {
        M->v[j] = w[j] / alpha - x[j];
        vd += M->v[j] * M->v[j] * M->D[j];
    }
    M->E = M->fval + 0.5 * mu * vd - lyap_theta(alpha) / (1.0 + alpha) * M->K;
    return M->E;
}

/* A new iterate (x, w) with column sums c; trace5 (may be NULL) receives
 * lhs1, rhs1, lhs2, rhs2, E of this iterate (NaN where there is no predecessor). */
static void mon_iterate(cond_mon *M, const double *x, const double *w, const double *c, const double *b,
                        double alpha, double mu, double fval, double *trace5)
{
    const int64_t m = M->m;
    double lhs1 = 0.0, lhs2 = 0.0, vd = 0.0, K = 0.0, l1 = 0.0;
    for (int64_t j = 0; j < m; j++) {
        double xi, D, Kj;
        metric_terms(c[j], b[j], &xi, &D, &Kj);
        const double v = w[j] / alpha - x[j];
        if (M->have) {
            lhs1 += M->xi[j] * M->xi[j] * D / (M->D[j] * M->D[j]);
            lhs2 += M->v[j] * M->v[j] * (D - M->D[j]);
        }
        vd += v * v * D;
        K += Kj;
        l1 += fabs(xi);
        M->xi[j] = xi;  /* the old values of column j are no longer needed */
        M->D[j] = D;
        M->v[j] = v;
    }
    const double E = fval + 0.5 * mu * vd - lyap_theta(alpha) / (1.0 + alpha) * K;
    double rhs1 = NAN, rhs2 = NAN;
    if (M->have) {
        rhs1 = (4.0 - alpha * alpha - 2.0 * sqrt(alpha)) / (2.0 * alpha * (1.0 + alpha) * (1.0 + alpha)) * M->K;
        rhs2 = pow(alpha, 1.5) * vd;
        if (!(lhs1 < rhs1)) M->n1++;
        if (!(lhs2 < rhs2)) M->n2++;
        if (E > M->E + 1e-8 + 1e-12 * fabs(fval) + 1e-6 * (0.5 * mu * vd + l1)) M->nl++;
    } else {
        lhs1 = lhs2 = NAN;
    }
    if (trace5) {
        trace5[0] = lhs1;
        trace5[1] = rhs1;
        trace5[2] = lhs2;
        trace5[3] = rhs2;
        trace5[4] = E;
    }
    M->K = K;
    M->E = E;
    M->fval = fval;
    M->have = 1;
}

/* Column sums c_j = exp(x_j + ell_j) of the plan at (u(x), x). */
static void col_sums(const double *x, const double *ell, int64_t m, double *c)
{
    for (int64_t j = 0; j < m; j++) c[j] = exp(x[j] + ell[j]);
}

/*
 * cond_counts (may be NULL; Acc only): [0] violations of condition 1, [1] of
 * condition 2, [2] Lyapunov rises, as the monitor above defines them.
 * trace_cond (may be NULL; length 5 (max_iter+1)): per It the monitor's
 * lhs1, rhs1, lhs2, rhs2, E.
 */
int oracle_solve_mon(int method, const double *C, int64_t n, int64_t m, double eps,
                     const double *a, const double *b, double tol, int64_t max_iter,
                     double mu0, int64_t m0, int w_rule, int restart,
                     double *f, double *g, int64_t *iters, int64_t *steps, double *err_out,
                     double *trace_err, double *trace_fval, double *trace_x,
                     int64_t *n_increase, int64_t *n_restart, int64_t *cond_counts, double *trace_cond)
{
    int64_t ninc = 0, nrst = 0;
    const int mon = method != ORACLE_SINKHORN && (cond_counts || trace_cond);
    cond_mon M;
    memset(&M, 0, sizeof(M));
    M.m = m;
    double *cs = NULL;
    if (mon) {
        M.xi = (double *)malloc(sizeof(double) * (size_t)m);
        M.D = (double *)malloc(sizeof(double) * (size_t)m);
        M.v = (double *)malloc(sizeof(double) * (size_t)m);
        cs = (double *)malloc(sizeof(double) * (size_t)m);
    }
    double *x = (double *)calloc((size_t)m, sizeof(double));
    double *w = (double *)calloc((size_t)m, sizeof(double));
    double *S = (double *)malloc(sizeof(double) * (size_t)m);
    double *ell = (double *)malloc(sizeof(double) * (size_t)m);
    double *u = (double *)malloc(sizeof(double) * (size_t)n);
    double err = 0.0, fval = 0.0;
    int64_t it = 0, nsteps = 0;
    int converged = 0;

    oracle_sstep(C, n, m, eps, a, b, x, u, ell, S, &err, &fval);
    nsteps = 1;
    double fprev = fval;
    if (trace_err) trace_err[0] = err;
    if (trace_fval) trace_fval[0] = fval;
    if (trace_x) memcpy(trace_x, x, sizeof(double) * (size_t)m);

    if (method == ORACLE_SINKHORN) {
        while (!(err < tol) && it < max_iter) {
            memcpy(x, S, sizeof(double) * (size_t)m);
            it++;
            oracle_sstep(C, n, m, eps, a, b, x, u, ell, S, &err, &fval);
            nsteps++;
            if (stability_increase(fval, fprev)) ninc++;
            fprev = fval;
            if (trace_err) trace_err[it] = err;
            if (trace_fval) trace_fval[it] = fval;
            if (trace_x) memcpy(trace_x + it * m, x, sizeof(double) * (size_t)m);
        }
    } else {
        double mu = mu0;
        int64_t mstage = m0;
        int done = (err < tol) || (it >= max_iter);
        if (mon) {  /* iterate 0: x_0 = w_0 = 0 */
            col_sums(x, ell, m, cs);
            mon_iterate(&M, x, w, cs, b, sqrt(2.0 * mu), mu, fval, trace_cond);
        }
        while (!done) {
            double alpha = sqrt(2.0 * mu);
            for (int64_t k = 0; k < mstage && !done; k++) {
                for (int64_t j = 0; j < m; j++) x[j] = (w[j] + S[j]) / (1.0 + alpha);
                oracle_sstep(C, n, m, eps, a, b, x, u, ell, S, &err, &fval);
                nsteps++;
                for (int64_t j = 0; j < m; j++)
                    w[j] = (w[j] + (alpha * alpha - 2.0) * x[j] + 2.0 * S[j]) / (1.0 + alpha);
                if (stability_increase(fval, fprev)) {
                    ninc++;
                    if (restart) {
                        for (int64_t j = 0; j < m; j++) w[j] = alpha * x[j];
                        nrst++;
                    }
                }
                fprev = fval;
                it++;
                if (mon) {
                    col_sums(x, ell, m, cs);
                    mon_iterate(&M, x, w, cs, b, alpha, mu, fval, trace_cond ? trace_cond + 5 * it : NULL);
                }
                if (trace_err) trace_err[it] = err;
                if (trace_fval) trace_fval[it] = fval;
                if (trace_x) memcpy(trace_x + it * m, x, sizeof(double) * (size_t)m);
                done = (err < tol) || (it >= max_iter);
            }
            if (!done) {
                double mu_new = mu / 2.0;
                if (w_rule == ORACLE_W_Y_CONTINUOUS) {
                    double ratio = sqrt(2.0 * mu_new) / alpha;
                    for (int64_t j = 0; j < m; j++) w[j] *= ratio;
                }
                mu = mu_new;
                mstage = (int64_t)floor(sqrt(2.0) * (double)mstage) + 1;
                if (mon) mon_rebase(&M, x, w, sqrt(2.0 * mu), mu);
            }
        }
    }
    if (cond_counts) {
        cond_counts[0] = mon ? M.n1 : -1;
        cond_counts[1] = mon ? M.n2 : -1;
        cond_counts[2] = mon ? M.nl : -1;
    }
    free(M.xi); free(M.D); free(M.v); free(cs);
    converged = err < tol;
    for (int64_t i = 0; i < n; i++) f[i] = eps * u[i];
    for (int64_t j = 0; j < m; j++) g[j] = eps * x[j];
    *iters = it;
    *steps = nsteps;
    *err_out = err;
    if (n_increase) *n_increase = ninc;
    if (n_restart) *n_restart = nrst;
    free(x); free(w); free(S); free(ell); free(u);
    return converged;
}

int oracle_solve_ex(int method, const double *C, int64_t n, int64_t m, double eps,
                    const double *a, const double *b, double tol, int64_t max_iter,
                    double mu0, int64_t m0, int w_rule, int restart,
                    double *f, double *g, int64_t *iters, int64_t *steps, double *err_out,
                    double *trace_err, double *trace_fval, double *trace_x,
                    int64_t *n_increase, int64_t *n_restart)
{
    return oracle_solve_mon(method, C, n, m, eps, a, b, tol, max_iter, mu0, m0, w_rule, restart, f, g, iters,
                            steps, err_out, trace_err, trace_fval, trace_x, n_increase, n_restart, NULL, NULL);
}

int oracle_solve(int method, const double *C, int64_t n, int64_t m, double eps,
                 const double *a, const double *b, double tol, int64_t max_iter,
                 double mu0, int64_t m0, int w_rule,
                 double *f, double *g, int64_t *iters, int64_t *steps, double *err_out,
                 double *trace_err, double *trace_fval, double *trace_x)
{
    return oracle_solve_ex(method, C, n, m, eps, a, b, tol, max_iter, mu0, m0, w_rule, 0, f, g, iters, steps,
                           err_out, trace_err, trace_fval, trace_x, NULL, NULL);
}

/*
 * Evaluation of given potentials (f, g) on cost C at eps, straight from the
 * definitions: P_ij = exp((f_i + g_j - C_ij)/eps) (eq:P-from-dual);
 * row_err = ||P1 - a||_1, col_err = ||P'1 - b||_1 (eq:l1tol);
 * dual = <f,a> + <g,b> - eps * sum_ij P_ij (the EOT dual value, eq:dual-obj
 * scaled back by eps); cost = <C,P>; mass = sum_ij P_ij.
 */
void oracle_eval(const double *C, int64_t n, int64_t m, double eps,
                 const double *a, const double *b, const double *f, const double *g,
                 double *row_err, double *col_err, double *dual, double *cost, double *mass)
{
    double *col = (double *)calloc((size_t)m, sizeof(double));
    double *rowsum = (double *)malloc(sizeof(double) * (size_t)n);
    double *rowcost = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double rs = 0.0, rc = 0.0;
        for (int64_t j = 0; j < m; j++) {
            double p = exp((f[i] + g[j] - C[i * m + j]) / eps);
            rs += p;
            rc += C[i * m + j] * p;
        }
        rowsum[i] = rs;
        rowcost[i] = rc;
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; j++) {
        double cs = 0.0;
        for (int64_t i = 0; i < n; i++) cs += exp((f[i] + g[j] - C[i * m + j]) / eps);
        col[j] = cs;
    }
    double re = 0.0, ce = 0.0, fa = 0.0, gb = 0.0, tot = 0.0, cst = 0.0;
    for (int64_t i = 0; i < n; i++) {
        re += fabs(rowsum[i] - a[i]);
        fa += f[i] * a[i];
        tot += rowsum[i];
        cst += rowcost[i];
    }
    for (int64_t j = 0; j < m; j++) {
        ce += fabs(col[j] - b[j]);
        gb += g[j] * b[j];
    }
    *row_err = re;
    *col_err = ce;
    *dual = fa + gb - eps * tot;
    *cost = cst;
    *mass = tot;
    free(col); free(rowsum); free(rowcost);
}

/*
 * The cost entry of two points, formed in FP64 from its definition (Sec. 5):
 * kind 0: ||x - y||^2 / scale (colour transfer), kind 1: (1 - <x, y>) / scale
 * (word alignment, unit rows).
 */
static double point_cost(int kind, const double *x, const double *y, int64_t d, double scale)
{
    double s = 0.0;
    if (kind == 0) {
        for (int64_t k = 0; k < d; k++) {
            double t = x[k] - y[k];
            s += t * t;
        }
        return s / scale;
    }
    for (int64_t k = 0; k < d; k++) s += x[k] * y[k];
    return (1.0 - s) / scale;
}

/*
 * oracle_eval on a point-cloud cost that is never stored: every C_ij is
 * formed from x_i and y_j when it is needed (once in the row pass, once in the
 * column pass), so problems far larger than an n x m array fit.  Same outputs
 * and definitions as oracle_eval (eq:P-from-dual, eq:l1tol, eq:dual-obj).
 */
void oracle_eval_points(int kind, const double *X, const double *Y, int64_t n, int64_t m, int64_t d,
                        double scale, double eps, const double *a, const double *b, const double *f,
                        const double *g, double *row_err, double *col_err, double *dual, double *cost,
                        double *mass)
{
    double *col = (double *)malloc(sizeof(double) * (size_t)m);
    double *rowsum = (double *)malloc(sizeof(double) * (size_t)n);
    double *rowcost = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        double rs = 0.0, rc = 0.0;
        for (int64_t j = 0; j < m; j++) {
            double c = point_cost(kind, X + i * d, Y + j * d, d, scale);
            double p = exp((f[i] + g[j] - c) / eps);
            rs += p;
            rc += c * p;
        }
        rowsum[i] = rs;
        rowcost[i] = rc;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < m; j++) {
        double cs = 0.0;
        for (int64_t i = 0; i < n; i++)
            cs += exp((f[i] + g[j] - point_cost(kind, X + i * d, Y + j * d, d, scale)) / eps);
        col[j] = cs;
    }
    double re = 0.0, ce = 0.0, fa = 0.0, gb = 0.0, tot = 0.0, cst = 0.0;
    for (int64_t i = 0; i < n; i++) {
        re += fabs(rowsum[i] - a[i]);
        fa += f[i] * a[i];
        tot += rowsum[i];
        cst += rowcost[i];
    }
    for (int64_t j = 0; j < m; j++) {
        ce += fabs(col[j] - b[j]);
        gb += g[j] * b[j];
    }
    *row_err = re;
    *col_err = ce;
    *dual = fa + gb - eps * tot;
    *cost = cst;
    *mass = tot;
    free(col); free(rowsum); free(rowcost);
}

/* Transport plan rows [row0, row0+rows): P_ij = exp((f_i + g_j - C_ij)/eps). */
void oracle_plan(const double *C, int64_t n, int64_t m, double eps,
                 const double *f, const double *g, int64_t row0, int64_t rows, double *P)
{
    (void)n;
    for (int64_t r = 0; r < rows; r++) {
        int64_t i = row0 + r;
        for (int64_t j = 0; j < m; j++) P[r * m + j] = exp((f[i] + g[j] - C[i * m + j]) / eps);
    }
}

/* Squared Euclidean cost C_ij = ||x_i - y_j||^2 / scale (Sec. 5, color transfer). */
void oracle_cost_sqeuclid(const double *X, const double *Y, int64_t n, int64_t m, int64_t d,
                          double scale, double *C)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = 0; j < m; j++) {
            double s = 0.0;
            for (int64_t k = 0; k < d; k++) {
                double t = X[i * d + k] - Y[j * d + k];
                s += t * t;
            }
            C[i * m + j] = s / scale;
        }
}

/* Cosine cost C_ij = (1 - <x_i, y_j>) / scale (Sec. 5, word alignment; rows of X, Y unit norm). */
void oracle_cost_cosine(const double *X, const double *Y, int64_t n, int64_t m, int64_t d,
                        double scale, double *C)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = 0; j < m; j++) {
            double s = 0.0;
            for (int64_t k = 0; k < d; k++) s += X[i * d + k] * Y[j * d + k];
            C[i * m + j] = (1.0 - s) / scale;
        }
}

/*
 * Gradients of the EOT value L(C) = <f,a> + <g,b> - eps*sum P at the optimum
 * with respect to the point clouds, by the envelope theorem: dL/dC_ij = P_ij.
 * kind 0 (squared Euclidean, C_ij = ||x_i - y_j||^2/scale):
 *   dL/dx_i = (2/scale) sum_j P_ij (x_i - y_j),  dL/dy_j = (2/scale) sum_i P_ij (y_j - x_i)
 * kind 1 (cosine, C_ij = (1 - x_i.y_j)/scale):
 *   dL/dx_i = -(1/scale) sum_j P_ij y_j,          dL/dy_j = -(1/scale) sum_i P_ij x_i
 * The plan P is formed from (f, g) on the exact FP64 cost.
 */
void oracle_grad_points(int kind, const double *X, const double *Y, int64_t n, int64_t m, int64_t d,
                        double scale, double eps, const double *f, const double *g,
                        double *dX, double *dY)
{
    double *C = (double *)malloc(sizeof(double) * (size_t)(n * m));
    if (kind == 0) oracle_cost_sqeuclid(X, Y, n, m, d, scale, C);
    else oracle_cost_cosine(X, Y, n, m, d, scale, C);
    memset(dX, 0, sizeof(double) * (size_t)(n * d));
    memset(dY, 0, sizeof(double) * (size_t)(m * d));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = 0; j < m; j++) {
            double p = exp((f[i] + g[j] - C[i * m + j]) / eps);
            for (int64_t k = 0; k < d; k++) {
                if (kind == 0) dX[i * d + k] += (2.0 / scale) * p * (X[i * d + k] - Y[j * d + k]);
                else dX[i * d + k] += -(1.0 / scale) * p * Y[j * d + k];
            }
        }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; j++)
        for (int64_t i = 0; i < n; i++) {
            double p = exp((f[i] + g[j] - C[i * m + j]) / eps);
            for (int64_t k = 0; k < d; k++) {
                if (kind == 0) dY[j * d + k] += (2.0 / scale) * p * (Y[j * d + k] - X[i * d + k]);
                else dY[j * d + k] += -(1.0 / scale) * p * X[i * d + k];
            }
        }
    free(C);
}
