/*
 * oci_oracle.h -- interface of the FP64 CPU oracle (test infrastructure only;
 * the product library neither includes nor links it).
 *
 * All arrays are host memory, float64, C order.  Shapes use J cells, N angles
 * (even), G groups, n = 4 N G:
 *   dx [J], sigma_t [J][G], sigma_s [J][G][G] with [j][g][gp] = gp -> g,
 *   speed [G], q [J][G][4], q_ang [J][G][N][4] (optional per-angle source),
 *   inc_l / inc_r [2][G][N/2] (levels k, k+1/2; NULL = vacuum),
 *   psi_prev [J][G][N][2], psi [J][G][N][4], phi [J][G][4].
 */
#ifndef OCI_ORACLE_H
#define OCI_ORACLE_H

enum {
    ORC_OK = 0,
    ORC_NOT_CONVERGED = 1,
    ORC_NONFINITE = 2,
    ORC_ERR_INVALID = -1,
    ORC_ERR_SINGULAR = -3,
};

enum { ORC_NORM_SCALAR = 0, ORC_NORM_ANGULAR = 1 };
enum { ORC_ORDER_JACOBI = 0, ORC_ORDER_RED_BLACK = 1 };

typedef struct {
    int J, N, G;
    const double *dx, *sigma_t, *sigma_s, *speed;
    double dt;
    int periodic;          /* test hook: 1 = periodic mesh instead of incident fluxes */
} orc_problem;

typedef struct {
    double tol;            /* epsilon of the rho_e stopping rule */
    int max_iters;         /* cap; reaching it reports ORC_NOT_CONVERGED */
    int fixed_iters;       /* > 0: run exactly this many iterations, no test */
    int norm;              /* ORC_NORM_SCALAR (default) or ORC_NORM_ANGULAR */
    int ordering;          /* ORC_ORDER_JACOBI (default) or ORC_ORDER_RED_BLACK */
} orc_control;

typedef struct {
    int iterations, status;
    double e_last, rho_e;
} orc_info;

int orc_gauss_legendre(int N, double *mu, double *w);
int orc_cell_matrix(const orc_problem *p, const double *mu, const double *w, int j, double *A);
int orc_lu_factor(int n, double *A, int *piv);
void orc_lu_solve(int n, const double *LU, const int *piv, double *b);

int orc_oci_setup(const orc_problem *p, double *lu, int *piv);
int orc_oci_iterate(const orc_problem *p, const double *lu, const int *piv,
                    const double *q, const double *q_ang, const double *psi_prev,
                    const double *inc_l, const double *inc_r,
                    const double *psi_in, double *psi_out);
int orc_oci_iterate_rb(const orc_problem *p, const double *lu, const int *piv,
                       const double *q, const double *q_ang, const double *psi_prev,
                       const double *inc_l, const double *inc_r,
                       const double *psi_in, double *psi_out);
int orc_oci_step(const orc_problem *p, const orc_control *c,
                 const double *lu, const int *piv,
                 const double *q, const double *q_ang,
                 const double *inc_l, const double *inc_r,
                 double *psi_prev, double *psi_iter, double *phi_out,
                 orc_info *info, double *e_hist);

int orc_si_setup(const orc_problem *p, double *lu4, int *piv4);
int orc_si_sweep(const orc_problem *p, const double *lu4, const int *piv4,
                 const double *q, const double *q_ang, const double *psi_prev,
                 const double *inc_l, const double *inc_r,
                 const double *phi_in, double *psi_out);
int orc_si_step(const orc_problem *p, const orc_control *c,
                const double *lu4, const int *piv4,
                const double *q, const double *q_ang,
                const double *inc_l, const double *inc_r,
                double *psi_prev, double *psi_iter, double *phi_out,
                orc_info *info, double *e_hist);

#endif
