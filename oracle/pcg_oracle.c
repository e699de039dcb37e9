/*
 * Oracle (test infrastructure only): preconditioned conjugate gradients for
 * the coarse Poisson systems K phi = b of Eqs. 12 and 15, in plain C.
 *
 * The paper solves these systems with GMRES(m)+ILU(0) (Section 2.3); K is
 * symmetric positive definite after homogeneous Dirichlet elimination, so the
 * oracle uses textbook preconditioned CG, and a mixed-precision variant: fp32 CG
 * refined by fp64 true residuals.  Stopping rule throughout: the true fp64
 * residual ||b - K phi||_2 <= tol * ||b||_2.
 *
 * Preconditioners: Jacobi, z = D^-1 r with D = diag(K) (deg <= 1), or a
 * Chebyshev polynomial in D^-1 K of degree deg (deg >= 2): z = the iterate after
 * deg steps of Chebyshev iteration for K z = r, preconditioned by D, from z = 0,
 * with the spectrum of D^-1 K taken to lie in [lo, hi] (textbook Chebyshev
 * acceleration).  For an eigenpair D^-1 K v = lam v it gives
 * z = s(lam) v for r = D v, where lam s(lam) = 1 - T_deg((c - lam)/e) / T_deg(c/e),
 * c = (hi + lo)/2, e = (hi - lo)/2; s > 0 on (0, hi], so the preconditioner is
 * symmetric positive definite when hi bounds the spectrum.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no fused multiply-add,
 * so every product and sum is rounded as written).
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

enum { ORACLE_OK = 0, ORACLE_NOCONV = 1, ORACLE_BREAKDOWN = 2 };

static void spmv64(int n, const int *rowptr, const int *col, const double *val,
                   const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) s += val[k] * x[col[k]];
        y[i] = s;
    }
}

static double dot64(int n, const double *a, const double *b) {
    double s = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : s)
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* threads an OpenMP region of this library runs with */
int oracle_threads(void) { return omp_get_max_threads(); }

void oracle_spmv_f64(int n, const int *rowptr, const int *col, const double *val,
                     const double *x, double *y) {
    spmv64(n, rowptr, col, val, x, y);
}

/* r = b - K x; returns ||r||_2 */
static double residual64(int n, const int *rowptr, const int *col, const double *val,
                         const double *b, const double *x, double *r) {
    spmv64(n, rowptr, col, val, x, r);
    double s = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : s)
    for (int i = 0; i < n; ++i) {
        r[i] = b[i] - r[i];
        s += r[i] * r[i];
    }
    return sqrt(s);
}

/* z = M^-1 r: Jacobi (deg <= 1) or the Chebyshev polynomial of degree deg; w1..w3 scratch [n] */
static void precond64(int n, const int *rowptr, const int *col, const double *val, const double *dinv,
                      int deg, double lo, double hi, const double *r, double *z, double *w1, double *w2,
                      double *w3) {
    if (deg <= 1) {
        for (int i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
        return;
    }
    const double c = 0.5 * (hi + lo), e = 0.5 * (hi - lo), sig = c / e;
    double rho = 1.0 / sig;
    double *res = w1, *d = w2, *t = w3;
    /* first step: z = D^-1 r / c */
    for (int i = 0; i < n; ++i) { d[i] = dinv[i] * r[i] / c; z[i] = d[i]; }
    spmv64(n, rowptr, col, val, z, res);
    for (int i = 0; i < n; ++i) res[i] = r[i] - res[i];
    for (int k = 1; k < deg; ++k) {
        const double rho_new = 1.0 / (2.0 * sig - rho);
        const double a1 = rho_new * rho, a2 = 2.0 * rho_new / e;
        for (int i = 0; i < n; ++i) { d[i] = a1 * d[i] + a2 * dinv[i] * res[i]; z[i] += d[i]; }
        if (k + 1 < deg) {   /* res -= K d (not needed after the last step) */
            spmv64(n, rowptr, col, val, d, t);
            for (int i = 0; i < n; ++i) res[i] -= t[i];
        }
        rho = rho_new;
    }
}

void oracle_cheb_apply_f64(int n, const int *rowptr, const int *col, const double *val, const double *dinv,
                           int deg, double lo, double hi, const double *r, double *z) {
    double *w1 = malloc(sizeof(double) * n), *w2 = malloc(sizeof(double) * n), *w3 = malloc(sizeof(double) * n);
    precond64(n, rowptr, col, val, dinv, deg, lo, hi, r, z, w1, w2, w3);
    free(w1); free(w2); free(w3);
}

/* the same in fp32 arithmetic with fp32 K (v32) and D^-1 (di32); coefficients rounded to fp32 */
static void precond32(int n, const int *rowptr, const int *col, const float *v32, const float *di32,
                      int deg, double lo, double hi, const float *r, float *z, float *w1, float *w2,
                      float *w3) {
    if (deg <= 1) {
        for (int i = 0; i < n; ++i) z[i] = di32[i] * r[i];
        return;
    }
    const double c = 0.5 * (hi + lo), e = 0.5 * (hi - lo), sig = c / e;
    double rho = 1.0 / sig;
    float *res = w1, *d = w2, *t = w3;
    const float ic = (float)(1.0 / c);
    for (int i = 0; i < n; ++i) { d[i] = di32[i] * r[i] * ic; z[i] = d[i]; }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        float acc = 0.0f;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) acc += v32[k] * z[col[k]];
        res[i] = r[i] - acc;
    }
    for (int k = 1; k < deg; ++k) {
        const double rho_new = 1.0 / (2.0 * sig - rho);
        const float a1 = (float)(rho_new * rho), a2 = (float)(2.0 * rho_new / e);
        for (int i = 0; i < n; ++i) { d[i] = a1 * d[i] + a2 * (di32[i] * res[i]); z[i] += d[i]; }
        if (k + 1 < deg) {
#pragma omp parallel for schedule(static)
            for (int i = 0; i < n; ++i) {
                float acc = 0.0f;
                for (int kk = rowptr[i]; kk < rowptr[i + 1]; ++kk) acc += v32[kk] * d[col[kk]];
                t[i] = acc;
            }
            for (int i = 0; i < n; ++i) res[i] -= t[i];
        }
        rho = rho_new;
    }
}

/*
 * fp64 PCG (preconditioner as above) from the guess held in x (overwritten with the solution).
 * When the recurrence residual meets the tolerance the true residual is
 * recomputed; if it does not meet it, CG restarts from the current iterate.
 * Returns ORACLE_OK / ORACLE_NOCONV (max_iter reached) / ORACLE_BREAKDOWN
 * (p.Kp <= 0 or a non-finite value).
 */
int oracle_pcg_f64(int n, const int *rowptr, const int *col, const double *val,
                   const double *dinv, int deg, double lo, double hi, const double *b, double *x,
                   double tol, int max_iter, int *iters_out, double *rel_res_out) {
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
    double *w1 = malloc(sizeof(double) * n), *w2 = malloc(sizeof(double) * n), *w3 = malloc(sizeof(double) * n);
    int status = ORACLE_NOCONV, it = 0;
    double bnorm = sqrt(dot64(n, b, b)), rnorm = 0.0;
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * n);
        status = ORACLE_OK;
        goto done;
    }
    rnorm = residual64(n, rowptr, col, val, b, x, r);
    if (!(rnorm == rnorm)) { status = ORACLE_BREAKDOWN; goto done; }
    while (rnorm > tol * bnorm) {
        /* (re)start: p = z = M^-1 r */
        precond64(n, rowptr, col, val, dinv, deg, lo, hi, r, z, w1, w2, w3);
        for (int i = 0; i < n; ++i) p[i] = z[i];
        double rho = dot64(n, r, z);
        for (;;) {
            if (it >= max_iter) { status = ORACLE_NOCONV; goto done; }
            spmv64(n, rowptr, col, val, p, q);
            double pq = dot64(n, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) { status = ORACLE_BREAKDOWN; goto done; }
            double alpha = rho / pq;
            for (int i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
            ++it;
            double rr = dot64(n, r, r);
            if (!isfinite(rr)) { status = ORACLE_BREAKDOWN; goto done; }
            if (sqrt(rr) <= tol * bnorm) break;
            precond64(n, rowptr, col, val, dinv, deg, lo, hi, r, z, w1, w2, w3);
            double rho_new = dot64(n, r, z);
            double beta = rho_new / rho;
            rho = rho_new;
            for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        }
        /* the recurrence says converged: check the true residual */
        rnorm = residual64(n, rowptr, col, val, b, x, r);
    }
    status = ORACLE_OK;
done:
    if (bnorm > 0.0) rnorm = residual64(n, rowptr, col, val, b, x, r);
    *iters_out = it;
    *rel_res_out = bnorm > 0.0 ? rnorm / bnorm : 0.0;
    free(r); free(z); free(p); free(q); free(w1); free(w2); free(w3);
    return status;
}

/*
 * Mixed precision: fp32 PCG whose residual is periodically replaced by
 * the true fp64 residual (iterative refinement by "reliable updates").
 *
 * The fp64 iterate x is only changed at a refinement step; between steps the
 * fp32 loop accumulates a correction c.  The fp32 recurrence residual r32 is
 * replaced by fl32(b - K x) (computed in fp64 after x += c) whenever ||r32||
 * has dropped below delta times its value at the previous refinement step, or
 * below the final tolerance.  A phase whose refinement point delta * s would
 * leave a short last phase (the tolerance within a factor delta^(1/4) of that
 * point) runs to the tolerance instead: refining there would cost a true
 * residual and a restart for a fraction of a phase.  The search direction p is kept across a
 * refinement step, so the Krylov information is not lost.  Convergence is
 * decided only on the true fp64 residual ||b - K x|| <= tol ||b||.  The inner
 * matrix (fl32 of K) and vectors are fp32; every dot product accumulates the
 * fp32 products in fp64.
 */
/* The value a refinement phase starting at true residual s measures its fall
 * against: s, or 0 (no refinement point, only the tolerance) when the point
 * delta * s is within a factor delta^(1/4) of the tolerance. */
static double phase_start(double s, double delta, double tol, double bnorm) {
    return delta * sqrt(sqrt(delta)) * s <= tol * bnorm ? 0.0 : s;
}

int oracle_pcg_mixed(int n, const int *rowptr, const int *col, const double *val,
                     const double *dinv, int deg, double lo, double hi, const double *b, double *x,
                     double tol, double delta, int max_iter, int *iters_out, int *updates_out,
                     double *rel_res_out) {
    int nnz = rowptr[n];
    float *v32 = malloc(sizeof(float) * nnz), *di32 = malloc(sizeof(float) * n);
    float *c = calloc((size_t)n, sizeof(float)), *r32 = malloc(sizeof(float) * n);
    float *z = malloc(sizeof(float) * n), *p = malloc(sizeof(float) * n);
    float *q = malloc(sizeof(float) * n);
    double *r = malloc(sizeof(double) * n);
    float *w1 = malloc(sizeof(float) * n), *w2 = malloc(sizeof(float) * n), *w3 = malloc(sizeof(float) * n);
    for (int k = 0; k < nnz; ++k) v32[k] = (float)val[k];
    for (int i = 0; i < n; ++i) di32[i] = (float)dinv[i];
    int status = ORACLE_NOCONV, it = 0, updates = 0;
    double bnorm = sqrt(dot64(n, b, b)), s = 0.0;
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * n);
        status = ORACLE_OK;
        goto done;
    }
    s = residual64(n, rowptr, col, val, b, x, r);
    if (!isfinite(s)) { status = ORACLE_BREAKDOWN; goto done; }
    if (s <= tol * bnorm) { status = ORACLE_OK; goto done; }
    double rho = 0.0, rmax = phase_start(s, delta, tol, bnorm);
    for (int i = 0; i < n; ++i) {
        r32[i] = (float)r[i];
        c[i] = 0.0f;
    }
    precond32(n, rowptr, col, v32, di32, deg, lo, hi, r32, z, w1, w2, w3);
    for (int i = 0; i < n; ++i) {
        p[i] = z[i];
        rho += (double)r32[i] * (double)z[i];
    }
    for (;;) {
        if (it >= max_iter) { status = ORACLE_NOCONV; goto done; }
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            float acc = 0.0f;
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) acc += v32[k] * p[col[k]];
            q[i] = acc;
        }
        double pq = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : pq)
        for (int i = 0; i < n; ++i) pq += (double)p[i] * (double)q[i];
        if (!(pq > 0.0) || !isfinite(pq)) { status = ORACLE_BREAKDOWN; goto done; }
        float alpha = (float)(rho / pq);
        double rsq = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : rsq)
        for (int i = 0; i < n; ++i) {
            c[i] += alpha * p[i];
            r32[i] -= alpha * q[i];
            rsq += (double)r32[i] * (double)r32[i];
        }
        ++it;
        double rn = sqrt(rsq);
        if (!isfinite(rn)) { status = ORACLE_BREAKDOWN; goto done; }
        if (rn <= delta * rmax || rn <= tol * bnorm) {
            /* refinement step: fold the fp32 correction into x, true fp64 residual */
            for (int i = 0; i < n; ++i) { x[i] += (double)c[i]; c[i] = 0.0f; }
            s = residual64(n, rowptr, col, val, b, x, r);
            ++updates;
            if (!isfinite(s)) { status = ORACLE_BREAKDOWN; goto done; }
            if (s <= tol * bnorm) { status = ORACLE_OK; goto done; }
            for (int i = 0; i < n; ++i) r32[i] = (float)r[i];
            rmax = phase_start(s, delta, tol, bnorm);
        }
        double rho_new = 0.0;
        precond32(n, rowptr, col, v32, di32, deg, lo, hi, r32, z, w1, w2, w3);
#pragma omp parallel for schedule(static) reduction(+ : rho_new)
        for (int i = 0; i < n; ++i) rho_new += (double)r32[i] * (double)z[i];
        float beta = (float)(rho_new / rho);
        rho = rho_new;
        for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
done:
    if (status != ORACLE_OK && bnorm > 0.0) {
        for (int i = 0; i < n; ++i) x[i] += (double)c[i];
    }
    s = bnorm > 0.0 ? residual64(n, rowptr, col, val, b, x, r) : 0.0;
    *iters_out = it;
    *updates_out = updates;
    *rel_res_out = bnorm > 0.0 ? s / bnorm : 0.0;
    free(v32); free(di32); free(c); free(r32); free(z); free(p); free(q); free(r);
    free(w1); free(w2); free(w3);
    return status;
}
