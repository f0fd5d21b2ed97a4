/*
 * oci_oracle.c -- plain FP64 CPU oracle for one-cell inversion (OCI) and
 * source iteration (SI) on the slab, multigroup, time-dependent S_N equations
 * discretised with simple corner balance (SCB) in space and multiple balance
 * (MB) in time.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code with the GPU path.
 *
 * Written for obviousness, not speed: dense per-cell matrices, textbook LU
 * with partial pivoting, and the iterations in the order the paper states
 * them.  OpenMP (when enabled) only spreads independent cells or independent
 * (group, angle) sweeps over threads; every reduction is summed serially in
 * ascending index order, so results do not depend on the thread count.
 *
 * Paper references (arXiv 2503.00264):
 *   transport equation ........ sec. 2.1, eq. (sn_nte)
 *   SCB + MB balances ......... sec. 2.1, eqs. (scb-mb-a..d) with the two closures
 *   OCI splitting ............. sec. 2.1, eq. (oci)
 *   within-cell operator ...... sec. 2.1, eqs. (Aja), (Aj)
 *   right-hand side ........... sec. 2.1, eq. (rhs_sg)
 *   scattering block .......... sec. 2.1, eq. (scatter); sec. 2.4, eq. (scatter_mg)
 *   unknown ordering .......... sec. 2.1, eq. (x_vec); sec. 2.4, eqs. (fullOCIlhs/rhs)
 *   stopping rule ............. sec. 2.1 (rho_e test); Algorithms 1 and 2
 *   SI cell system ............ Appendix A, eqs. (si_sys), (si_rhs), (si_sf)
 *
 * Readings where the paper is garbled or silent (each is listed in the
 * design notes):
 *   R1 scattering block: entry ((g,m,u),(g',n,u')) = dx*Ss[g'->g]/4 * w_n when
 *      u == u' (same corner and time level), zero otherwise; this is what the
 *      scalar flux phi = sum_n w_n psi_n inside the balances produces.
 *   R2 every group uses its own total cross section and speed in L_c.
 *   R3 the first iterate of a time step is the last iterate of the previous
 *      step (all four components); before the first step it is the initial
 *      angular flux copied to both time levels.  SI's first lagged scalar flux
 *      is the one of that iterate.
 *   R4 the rho_e test is applied from the second iteration on; e == 0 counts
 *      as converged; a cap on iterations reports "not converged".
 *   R5 the default convergence norm is the L2 norm of the change in scalar
 *      flux over every (cell, group, corner, time level); the angular-flux
 *      norm of Algorithm 2 is an option.
 *   R6 SI couples groups by Jacobi iteration: the whole scattering source
 *      sum_g' Ss[g'->g] phi_g' is taken from the previous iterate.
 *
 * Unknown layout (eq. x_vec, multigroup group-major): index of
 * (group g, angle m, component u) in a cell is (g*N + m)*4 + u with
 * u = 0: psi_{k,L}, 1: psi_{k,R}, 2: psi_{k+1/2,L}, 3: psi_{k+1/2,R}.
 * Angles are Gauss-Legendre nodes in ascending order (mu < 0 first).
 */
#include "oci_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IDX4(p, j, g, m, u) ((((size_t)(j) * (p)->G + (g)) * (p)->N + (m)) * 4 + (u))
#define IDX2(p, j, g, m, c) ((((size_t)(j) * (p)->G + (g)) * (p)->N + (m)) * 2 + (c))

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre quadrature (footnote of the introduction: GL is used for   */
/* every result).  Newton's method on P_N from the Chebyshev-like guess      */
/* cos(pi (i + 3/4) / (N + 1/2)); weights 2 / ((1 - x^2) P_N'(x)^2).          */
/* ------------------------------------------------------------------------ */
static void legendre_pn(int N, double x, double *pn, double *dpn)
{
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= N; ++k) {
        double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
    }
    *pn = p1;
    *dpn = N * (x * p1 - p0) / (x * x - 1.0);
}

int orc_gauss_legendre(int N, double *mu, double *w)
{
    if (N < 2 || (N & 1)) return ORC_ERR_INVALID;
    for (int i = 0; i < N; ++i) {
        double x = cos(M_PI * (i + 0.75) / (N + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre_pn(N, x, &p, &dp);
            double step = p / dp;
            x -= step;
            if (fabs(step) < 1e-16) break;
        }
        double p, dp;
        legendre_pn(N, x, &p, &dp);
        /* i = 0 is the largest root; store ascending */
        mu[N - 1 - i] = x;
        w[N - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Problem validation                                                        */
/* ------------------------------------------------------------------------ */
static int check_problem(const orc_problem *p)
{
    if (!p || p->J < 1 || p->G < 1 || p->N < 2 || (p->N & 1)) return ORC_ERR_INVALID;
    if (!p->dx || !p->sigma_t || !p->sigma_s || !p->speed) return ORC_ERR_INVALID;
    if (!(p->dt > 0.0)) return ORC_ERR_INVALID;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Cell matrix A_j (eqs. Aja, Aj, scatter, fullOCIlhs).                      */
/* Row-major n x n, n = 4 N G.                                               */
/* ------------------------------------------------------------------------ */
int orc_cell_matrix(const orc_problem *p, const double *mu, const double *w,
                    int j, double *A)
{
    int rc = check_problem(p);
    if (rc) return rc;
    const int N = p->N, G = p->G, n = 4 * N * G;
    const double dx = p->dx[j];
    memset(A, 0, sizeof(double) * (size_t)n * n);

    /* block-diagonal within-cell operator L_{c,j,g,m} (eq. Aj) */
    for (int g = 0; g < G; ++g) {
        const double sig = p->sigma_t[(size_t)j * G + g];
        const double a = dx / (p->speed[g] * p->dt);          /* dx / (v dt) */
        for (int m = 0; m < N; ++m) {
            const double d = 0.5 * (fabs(mu[m]) + dx * sig);  /* (|mu| + dx Sigma)/2 */
            const double h = 0.5 * mu[m];                      /* mu / 2 */
            const int b = (g * N + m) * 4;
            double *r0 = A + (size_t)(b + 0) * n + b;
            double *r1 = A + (size_t)(b + 1) * n + b;
            double *r2 = A + (size_t)(b + 2) * n + b;
            double *r3 = A + (size_t)(b + 3) * n + b;
            r0[0] = d;      r0[1] = h;      r0[2] = 0.5 * a; r0[3] = 0.0;
            r1[0] = -h;     r1[1] = d;      r1[2] = 0.0;     r1[3] = 0.5 * a;
            r2[0] = -a;     r2[1] = 0.0;    r2[2] = a + d;   r2[3] = h;
            r3[0] = 0.0;    r3[1] = -a;     r3[2] = -h;      r3[3] = a + d;
        }
    }
    /* minus the scattering blocks S_{g'->g,j} (reading R1) */
    for (int g = 0; g < G; ++g)
        for (int gp = 0; gp < G; ++gp) {
            const double s = 0.25 * dx * p->sigma_s[((size_t)j * G + g) * G + gp];
            for (int m = 0; m < N; ++m)
                for (int nn = 0; nn < N; ++nn)
                    for (int u = 0; u < 4; ++u) {
                        const int r = (g * N + m) * 4 + u;
                        const int c = (gp * N + nn) * 4 + u;
                        A[(size_t)r * n + c] -= s * w[nn];
                    }
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* LU with partial pivoting (the factorisation a general dense solver such   */
/* as LAPACK's gesv performs; sec. 2.5).  Pivot = largest |a_ik|, the lowest */
/* row index winning ties.  A is overwritten by the unit-lower L (below the  */
/* diagonal) and U; piv[k] is the row exchanged with row k.                  */
/* ------------------------------------------------------------------------ */
int orc_lu_factor(int n, double *A, int *piv)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(A[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = fabs(A[(size_t)i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        piv[k] = p;
        if (best == 0.0) return ORC_ERR_SINGULAR;
        if (p != k)
            for (int c = 0; c < n; ++c) {
                double t = A[(size_t)k * n + c];
                A[(size_t)k * n + c] = A[(size_t)p * n + c];
                A[(size_t)p * n + c] = t;
            }
        const double pivot = A[(size_t)k * n + k];
        for (int i = k + 1; i < n; ++i) {
            double l = A[(size_t)i * n + k] / pivot;
            A[(size_t)i * n + k] = l;
            for (int c = k + 1; c < n; ++c)
                A[(size_t)i * n + c] -= l * A[(size_t)k * n + c];
        }
    }
    return ORC_OK;
}

/* Forward then backward substitution with the factors (LAPACK getrs). */
void orc_lu_solve(int n, const double *LU, const int *piv, double *b)
{
    for (int k = 0; k < n; ++k) {
        int p = piv[k];
        if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; }
    }
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= LU[(size_t)i * n + k] * b[k];
        b[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int k = i + 1; k < n; ++k) s -= LU[(size_t)i * n + k] * b[k];
        b[i] = s / LU[(size_t)i * n + i];
    }
}

/* ------------------------------------------------------------------------ */
/* Upstream edge values seen by cell j (the upstream closure of sec. 2.1).   */
/* For mu_m > 0 the flux entering at the left edge of cell j, at time level   */
/* lev (0: k, 1: k+1/2): the right corner of cell j-1, or the prescribed     */
/* incident flux at x = 0.  For mu_m < 0, the flux entering at the right     */
/* edge: the left corner of cell j+1, or the incident flux at x = X.         */
/* `psi` is the angular flux iterate [J][G][N][4].                           */
/* ------------------------------------------------------------------------ */
static double upstream_edge(const orc_problem *p, const double *mu, const double *psi,
                            const double *inc_l, const double *inc_r,
                            int j, int g, int m, int lev)
{
    const int N = p->N, G = p->G, J = p->J, half = N / 2;
    if (mu[m] > 0.0) {
        int jn = j - 1;
        if (jn < 0) {
            if (!p->periodic)
                return inc_l ? inc_l[((size_t)lev * G + g) * half + (m - half)] : 0.0;
            jn = J - 1;
        }
        return psi[IDX4(p, jn, g, m, lev == 0 ? 1 : 3)];
    } else {
        int jn = j + 1;
        if (jn >= J) {
            if (!p->periodic)
                return inc_r ? inc_r[((size_t)lev * G + g) * half + m] : 0.0;
            jn = 0;
        }
        return psi[IDX4(p, jn, g, m, lev == 0 ? 0 : 2)];
    }
}

/* Source and previous-time terms of b_{j,g,m} (eq. rhs_sg without the      */
/* incident part).  The isotropic source enters as dx/4 * Q; the optional   */
/* per-angle source hook q_ang (angular density, same four components)      */
/* replaces it by dx/2 * q_ang.                                              */
static void const_rhs(const orc_problem *p, const double *q, const double *q_ang,
                      const double *psi_prev, int j, int g, int m, double out[4])
{
    const double dx = p->dx[j];
    const double a2 = dx / (2.0 * p->speed[g] * p->dt);     /* dx / (2 v dt) */
    for (int u = 0; u < 4; ++u) {
        if (q_ang)
            out[u] = 0.5 * dx * q_ang[IDX4(p, j, g, m, u)];
        else
            out[u] = q ? 0.25 * dx * q[((size_t)j * p->G + g) * 4 + u] : 0.0;
    }
    out[0] += a2 * psi_prev[IDX2(p, j, g, m, 0)];
    out[1] += a2 * psi_prev[IDX2(p, j, g, m, 1)];
}

/* Full b_j for the OCI system from the iterate psi (eq. rhs_sg, fullOCIrhs). */
static void oci_rhs(const orc_problem *p, const double *mu, const double *q,
                    const double *q_ang, const double *psi_prev,
                    const double *inc_l, const double *inc_r,
                    const double *psi, int j, double *b)
{
    for (int g = 0; g < p->G; ++g)
        for (int m = 0; m < p->N; ++m) {
            double c[4];
            const_rhs(p, q, q_ang, psi_prev, j, g, m, c);
            const double ek = upstream_edge(p, mu, psi, inc_l, inc_r, j, g, m, 0);
            const double eh = upstream_edge(p, mu, psi, inc_l, inc_r, j, g, m, 1);
            if (mu[m] > 0.0) {           /* b^+ : incident through the left edge */
                c[0] += mu[m] * ek;
                c[2] += mu[m] * eh;
            } else {                     /* b^- : incident through the right edge */
                c[1] -= mu[m] * ek;
                c[3] -= mu[m] * eh;
            }
            double *bb = b + (size_t)(g * p->N + m) * 4;
            bb[0] = c[0]; bb[1] = c[1]; bb[2] = c[2]; bb[3] = c[3];
        }
}

/* ------------------------------------------------------------------------ */
/* Setup: assemble every A_j and factor it (Algorithm 2, first line; the    */
/* l = 0 gesv of the loop).  lu [J][n][n], piv [J][n].                       */
/* ------------------------------------------------------------------------ */
int orc_oci_setup(const orc_problem *p, double *lu, int *piv)
{
    int rc = check_problem(p);
    if (rc) return rc;
    const int n = 4 * p->N * p->G;
    double *mu = malloc(sizeof(double) * p->N), *w = malloc(sizeof(double) * p->N);
    orc_gauss_legendre(p->N, mu, w);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|:bad)
    for (int j = 0; j < p->J; ++j) {
        double *A = lu + (size_t)j * n * n;
        orc_cell_matrix(p, mu, w, j, A);
        if (orc_lu_factor(n, A, piv + (size_t)j * n)) bad |= 1;
    }
    free(mu);
    free(w);
    return bad ? ORC_ERR_SINGULAR : ORC_OK;
}

/* One OCI (cell-wise block Jacobi) iteration, eq. (oci): every cell solves   */
/* its own system with the incident edges taken from psi_in only.            */
int orc_oci_iterate(const orc_problem *p, const double *lu, const int *piv,
                    const double *q, const double *q_ang, const double *psi_prev,
                    const double *inc_l, const double *inc_r,
                    const double *psi_in, double *psi_out)
{
    int rc = check_problem(p);
    if (rc) return rc;
    const int n = 4 * p->N * p->G;
    double *mu = malloc(sizeof(double) * p->N), *w = malloc(sizeof(double) * p->N);
    orc_gauss_legendre(p->N, mu, w);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < p->J; ++j) {
        double *b = psi_out + (size_t)j * n;
        oci_rhs(p, mu, q, q_ang, psi_prev, inc_l, inc_r, psi_in, j, b);
        orc_lu_solve(n, lu + (size_t)j * n * n, piv + (size_t)j * n, b);
    }
    free(mu);
    free(w);
    return ORC_OK;
}

/* One red-black OCI iteration (the cell-wise block Gauss-Seidel ordering     */
/* the paper names beside block Jacobi in its introduction): the even         */
/* ("red") cells solve first with their incident edges from psi_in; then the  */
/* odd ("black") cells solve with the edges of their red neighbours just      */
/* computed.  Each cell's solve is the same as in orc_oci_iterate; only the   */
/* iterate its upstream edges come from differs.                              */
int orc_oci_iterate_rb(const orc_problem *p, const double *lu, const int *piv,
                       const double *q, const double *q_ang, const double *psi_prev,
                       const double *inc_l, const double *inc_r,
                       const double *psi_in, double *psi_out)
{
    int rc = check_problem(p);
    if (rc) return rc;
    const int n = 4 * p->N * p->G;
    double *mu = malloc(sizeof(double) * p->N), *w = malloc(sizeof(double) * p->N);
    orc_gauss_legendre(p->N, mu, w);
    for (int colour = 0; colour < 2; ++colour) {
        const double *src = colour == 0 ? psi_in : psi_out;
#pragma omp parallel for schedule(static)
        for (int j = colour; j < p->J; j += 2) {
            double *b = psi_out + (size_t)j * n;
            oci_rhs(p, mu, q, q_ang, psi_prev, inc_l, inc_r, src, j, b);
            orc_lu_solve(n, lu + (size_t)j * n * n, piv + (size_t)j * n, b);
        }
    }
    free(mu);
    free(w);
    return ORC_OK;
}

/* Scalar flux phi_{j,g,u} = sum_m w_m psi_{j,g,m,u} (eq. si_sf); [J][G][4]. */
static void scalar_flux(const orc_problem *p, const double *w, const double *psi, double *phi)
{
    for (int j = 0; j < p->J; ++j)
        for (int g = 0; g < p->G; ++g)
            for (int u = 0; u < 4; ++u) {
                double s = 0.0;
                for (int m = 0; m < p->N; ++m) s += w[m] * psi[IDX4(p, j, g, m, u)];
                phi[((size_t)j * p->G + g) * 4 + u] = s;
            }
}

/* L2 norm of a difference, summed in ascending index order. */
static double diff_norm(size_t len, const double *a, const double *b)
{
    double s = 0.0;
    for (size_t i = 0; i < len; ++i) {
        double d = a[i] - b[i];
        s += d * d;
    }
    return sqrt(s);
}

/* Stopping rule (sec. 2.1 and Algorithms 1/2, readings R4): returns 1 when   */
/* the iteration stops after `iters` iterations with change e.               */
static int stop_rule(const orc_control *c, int iters, double e, double e_prev,
                     orc_info *info)
{
    info->iterations = iters;
    info->e_last = e;
    info->rho_e = iters >= 2 ? e / e_prev : NAN;
    if (!isfinite(e)) { info->status = ORC_NONFINITE; return 1; }
    if (c->fixed_iters > 0) {
        info->status = ORC_OK;
        return iters >= c->fixed_iters;
    }
    if (iters >= 2) {
        if (e == 0.0) { info->status = ORC_OK; return 1; }
        if (e < c->tol * (1.0 - e / e_prev)) { info->status = ORC_OK; return 1; }
    }
    if (iters >= c->max_iters) { info->status = ORC_NOT_CONVERGED; return 1; }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One OCI time step (Algorithm 2).  psi_iter [J][G][N][4] holds the first   */
/* iterate on entry (reading R3) and the last iterate on exit; psi_prev      */
/* [J][G][N][2] holds psi_{k-1/2} on entry and psi_{k+1/2} on exit (the time */
/* update).  phi_out [J][G][4] receives the scalar flux of the last iterate. */
/* e_hist (optional, >= max_iters or fixed_iters entries) receives e_l.      */
/* ------------------------------------------------------------------------ */
int orc_oci_step(const orc_problem *p, const orc_control *c,
                 const double *lu, const int *piv,
                 const double *q, const double *q_ang,
                 const double *inc_l, const double *inc_r,
                 double *psi_prev, double *psi_iter, double *phi_out,
                 orc_info *info, double *e_hist)
{
    int rc = check_problem(p);
    if (rc) return rc;
    if (!c || !info || !psi_prev || !psi_iter) return ORC_ERR_INVALID;
    if (c->fixed_iters <= 0 && (c->max_iters < 1 || !(c->tol >= 0.0))) return ORC_ERR_INVALID;
    const int N = p->N, G = p->G;
    const size_t len = (size_t)p->J * G * N * 4, flen = (size_t)p->J * G * 4;
    double *mu = malloc(sizeof(double) * N), *w = malloc(sizeof(double) * N);
    orc_gauss_legendre(N, mu, w);
    double *next = malloc(sizeof(double) * len);
    double *phi_old = malloc(sizeof(double) * flen), *phi_new = malloc(sizeof(double) * flen);
    scalar_flux(p, w, psi_iter, phi_old);

    double e_prev = NAN;
    int iters = 0;
    memset(info, 0, sizeof(*info));
    for (;;) {
        if (c->ordering == ORC_ORDER_RED_BLACK)
            orc_oci_iterate_rb(p, lu, piv, q, q_ang, psi_prev, inc_l, inc_r, psi_iter, next);
        else
            orc_oci_iterate(p, lu, piv, q, q_ang, psi_prev, inc_l, inc_r, psi_iter, next);
        scalar_flux(p, w, next, phi_new);
        double e = c->norm == ORC_NORM_ANGULAR ? diff_norm(len, next, psi_iter)
                                               : diff_norm(flen, phi_new, phi_old);
        if (e_hist) e_hist[iters] = e;
        ++iters;
        memcpy(psi_iter, next, sizeof(double) * len);
        memcpy(phi_old, phi_new, sizeof(double) * flen);
        if (stop_rule(c, iters, e, e_prev, info)) break;
        e_prev = e;
    }
    /* end of step: psi_{k-1/2} <- psi_{k+1/2} (sec. 2.1, after convergence) */
    for (int j = 0; j < p->J; ++j)
        for (int g = 0; g < G; ++g)
            for (int m = 0; m < N; ++m) {
                psi_prev[IDX2(p, j, g, m, 0)] = psi_iter[IDX4(p, j, g, m, 2)];
                psi_prev[IDX2(p, j, g, m, 1)] = psi_iter[IDX4(p, j, g, m, 3)];
            }
    if (phi_out) memcpy(phi_out, phi_old, sizeof(double) * flen);
    free(mu); free(w); free(next); free(phi_old); free(phi_new);
    return info->status;
}

/* ------------------------------------------------------------------------ */
/* Source iteration (Appendix A, Algorithm 1).                               */
/* ------------------------------------------------------------------------ */

/* The 4x4 SI cell matrix of (g, m) in cell j: the L_{c,j,g,m} of eq. (Aj). */
static void si_cell_matrix(const orc_problem *p, const double *mu, int j, int g, int m,
                           double L[16])
{
    const double dx = p->dx[j];
    const double sig = p->sigma_t[(size_t)j * p->G + g];
    const double a = dx / (p->speed[g] * p->dt);
    const double d = 0.5 * (fabs(mu[m]) + dx * sig), h = 0.5 * mu[m];
    const double M[16] = {d, h, 0.5 * a, 0.0,
                          -h, d, 0.0, 0.5 * a,
                          -a, 0.0, a + d, h,
                          0.0, -a, -h, a + d};
    memcpy(L, M, sizeof(M));
}

/* One SI transport sweep for angle m of group g with the lagged scalar flux  */
/* phi [J][G][4]: mu > 0 sweeps j = 0..J-1, mu < 0 sweeps j = J-1..0, each   */
/* cell solving its 4x4 system with the upstream value just computed.  On a  */
/* periodic mesh the wrap-around edge is found by superposition: the sweep   */
/* is affine in the two entering edge values, so three sweeps give the map   */
/* and a 2x2 solve closes the ring.                                          */
static void si_sweep_one(const orc_problem *p, const double *mu, const double *q,
                         const double *q_ang, const double *psi_prev,
                         const double *inc_l, const double *inc_r,
                         const double *phi, const double *lu4, const int *piv4,
                         int g, int m, double *psi_out)
{
    const int J = p->J, G = p->G, N = p->N, half = N / 2;
    const int pos = mu[m] > 0.0;

    /* sweep with given entering edge values (level k, level k+1/2); returns
     * the leaving edge values after the last cell */
    #define SWEEP(E0, E1, OUT0, OUT1, SRC_ON)                                        \
    do {                                                                             \
        double e0 = (E0), e1 = (E1);                                                 \
        for (int s = 0; s < J; ++s) {                                                \
            const int j = pos ? s : J - 1 - s;                                       \
            double d[4] = {0, 0, 0, 0};                                              \
            if (SRC_ON) {                                                            \
                const_rhs(p, q, q_ang, psi_prev, j, g, m, d);                        \
                for (int u = 0; u < 4; ++u) {                                        \
                    double sc = 0.0;                                                 \
                    for (int gp = 0; gp < G; ++gp)                                   \
                        sc += p->sigma_s[((size_t)j * G + g) * G + gp] *             \
                              phi[((size_t)j * G + gp) * 4 + u];                     \
                    d[u] += 0.25 * p->dx[j] * sc;                                    \
                }                                                                    \
            }                                                                        \
            if (pos) { d[0] += mu[m] * e0; d[2] += mu[m] * e1; }                     \
            else     { d[1] -= mu[m] * e0; d[3] -= mu[m] * e1; }                     \
            const size_t k4 = (((size_t)j * G + g) * N + m);                         \
            orc_lu_solve(4, lu4 + k4 * 16, piv4 + k4 * 4, d);                        \
            for (int u = 0; u < 4; ++u) psi_out[IDX4(p, j, g, m, u)] = d[u];         \
            e0 = pos ? d[1] : d[0];                                                  \
            e1 = pos ? d[3] : d[2];                                                  \
        }                                                                            \
        OUT0 = e0; OUT1 = e1;                                                        \
    } while (0)

    double in0, in1;
    if (!p->periodic) {
        if (pos) {
            in0 = inc_l ? inc_l[((size_t)0 * G + g) * half + (m - half)] : 0.0;
            in1 = inc_l ? inc_l[((size_t)1 * G + g) * half + (m - half)] : 0.0;
        } else {
            in0 = inc_r ? inc_r[((size_t)0 * G + g) * half + m] : 0.0;
            in1 = inc_r ? inc_r[((size_t)1 * G + g) * half + m] : 0.0;
        }
    } else {
        double z0, z1, a0, a1, b0, b1;
        SWEEP(0.0, 0.0, z0, z1, 1);   /* affine part */
        SWEEP(1.0, 0.0, a0, a1, 0);   /* response to a unit level-k edge */
        SWEEP(0.0, 1.0, b0, b1, 0);   /* response to a unit level-k+1/2 edge */
        /* solve x = z + [a b] x for the wrap-around edge x */
        const double m00 = 1.0 - a0, m01 = -b0, m10 = -a1, m11 = 1.0 - b1;
        const double det = m00 * m11 - m01 * m10;
        in0 = (m11 * z0 - m01 * z1) / det;
        in1 = (-m10 * z0 + m00 * z1) / det;
    }
    double o0, o1;
    SWEEP(in0, in1, o0, o1, 1);
    (void)o0; (void)o1;
    #undef SWEEP
}

/* SI setup: the 4x4 LU factors of every L_{c,j,g,m} (the l = 0 gesv of      */
/* Algorithm 1).  lu4 [J][G][N][16], piv4 [J][G][N][4].                       */
int orc_si_setup(const orc_problem *p, double *lu4, int *piv4)
{
    int rc = check_problem(p);
    if (rc) return rc;
    double *mu = malloc(sizeof(double) * p->N), *w = malloc(sizeof(double) * p->N);
    orc_gauss_legendre(p->N, mu, w);
    int bad = 0;
    for (int j = 0; j < p->J; ++j)
        for (int g = 0; g < p->G; ++g)
            for (int m = 0; m < p->N; ++m) {
                const size_t k = ((size_t)j * p->G + g) * p->N + m;
                si_cell_matrix(p, mu, j, g, m, lu4 + k * 16);
                if (orc_lu_factor(4, lu4 + k * 16, piv4 + k * 4)) bad = 1;
            }
    free(mu);
    free(w);
    return bad ? ORC_ERR_SINGULAR : ORC_OK;
}

/* One SI iteration: every (g, m) sweep with the lagged scalar flux phi_in. */
int orc_si_sweep(const orc_problem *p, const double *lu4, const int *piv4,
                 const double *q, const double *q_ang, const double *psi_prev,
                 const double *inc_l, const double *inc_r,
                 const double *phi_in, double *psi_out)
{
    int rc = check_problem(p);
    if (rc) return rc;
    double *mu = malloc(sizeof(double) * p->N), *w = malloc(sizeof(double) * p->N);
    orc_gauss_legendre(p->N, mu, w);
    const int GN = p->G * p->N;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < GN; ++k)
        si_sweep_one(p, mu, q, q_ang, psi_prev, inc_l, inc_r, phi_in, lu4, piv4,
                     k / p->N, k % p->N, psi_out);
    free(mu);
    free(w);
    return ORC_OK;
}

/* One SI time step (Algorithm 1, readings R3-R6).  Same state convention as */
/* orc_oci_step: psi_iter is the previous step's last angular flux on entry  */
/* (its scalar flux is the first lagged source) and the last sweep on exit.  */
int orc_si_step(const orc_problem *p, const orc_control *c,
                const double *lu4, const int *piv4,
                const double *q, const double *q_ang,
                const double *inc_l, const double *inc_r,
                double *psi_prev, double *psi_iter, double *phi_out,
                orc_info *info, double *e_hist)
{
    int rc = check_problem(p);
    if (rc) return rc;
    if (!c || !info || !psi_prev || !psi_iter) return ORC_ERR_INVALID;
    if (c->fixed_iters <= 0 && (c->max_iters < 1 || !(c->tol >= 0.0))) return ORC_ERR_INVALID;
    const int N = p->N, G = p->G;
    const size_t flen = (size_t)p->J * G * 4;
    double *mu = malloc(sizeof(double) * N), *w = malloc(sizeof(double) * N);
    orc_gauss_legendre(N, mu, w);
    double *phi_old = malloc(sizeof(double) * flen), *phi_new = malloc(sizeof(double) * flen);
    scalar_flux(p, w, psi_iter, phi_old);

    double e_prev = NAN;
    int iters = 0;
    memset(info, 0, sizeof(*info));
    for (;;) {
        orc_si_sweep(p, lu4, piv4, q, q_ang, psi_prev, inc_l, inc_r, phi_old, psi_iter);
        scalar_flux(p, w, psi_iter, phi_new);
        double e = diff_norm(flen, phi_new, phi_old);
        if (e_hist) e_hist[iters] = e;
        ++iters;
        memcpy(phi_old, phi_new, sizeof(double) * flen);
        if (stop_rule(c, iters, e, e_prev, info)) break;
        e_prev = e;
    }
    for (int j = 0; j < p->J; ++j)
        for (int g = 0; g < G; ++g)
            for (int m = 0; m < N; ++m) {
                psi_prev[IDX2(p, j, g, m, 0)] = psi_iter[IDX4(p, j, g, m, 2)];
                psi_prev[IDX2(p, j, g, m, 1)] = psi_iter[IDX4(p, j, g, m, 3)];
            }
    if (phi_out) memcpy(phi_out, phi_old, sizeof(double) * flen);
    free(mu); free(w); free(phi_old); free(phi_new);
    return info->status;
}
