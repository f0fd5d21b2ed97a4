/*
 * oci.h -- C ABI of liboci, the MI355X (gfx950) one-cell-inversion library for
 * slab-geometry, multigroup, time-dependent discrete-ordinates (S_N) transport
 * with simple-corner-balance (SCB) space and multiple-balance (MB) time
 * discretisation (arXiv 2503.00264).
 *
 * What is computed (paper section 2):
 *   The unknowns of cell j are the angular fluxes psi_{g,m,u} for group g,
 *   Gauss-Legendre angle m and component u = 0: (k,L), 1: (k,R),
 *   2: (k+1/2,L), 3: (k+1/2,R) (eq. x_vec, group-major as in eqs.
 *   fullOCIlhs/fullOCIrhs); n = 4 N G unknowns per cell.  They satisfy the four
 *   corner balances (eqs. scb-mb-a..d) with the midpoint closure and the
 *   upstream edge closure.
 *   oci_step performs one time step with the one-cell-inversion iteration of
 *   eq. (oci): every cell solves A_j Psi_j^(l+1) = b_j(Psi^(l)) with
 *   A_j = blockdiag(L_c) - S (eqs. Aj, scatter, scatter_mg, fullOCIlhs) and
 *   b_j from eq. (rhs_sg), the incident edge fluxes lagged (block Jacobi over
 *   cells), until the stopping rule of section 2.1 holds.
 *   si_step performs the same time step with source iteration (Appendix A:
 *   eqs. si_sys, si_rhs, si_sf; Algorithm 1), all groups and angles swept in
 *   parallel with the whole scattering source lagged (Jacobi in groups).
 *
 * Stopping rule (section 2.1; Algorithms 1 and 2): after iteration l >= 1,
 *   stop when e_l < tol (1 - e_l / e_{l-1}), e_l = ||x^(l+1) - x^(l)||_2 over
 *   every (cell, group, corner, time level) of the scalar flux
 *   phi = sum_m w_m psi_m (OCI_NORM_SCALAR; SI always uses it) or of the
 *   angular flux (OCI_NORM_ANGULAR, Algorithm 2).  e_l == 0 stops.  Reaching
 *   max_iters stops with OCI_NOT_CONVERGED; a non-finite e_l stops with
 *   OCI_NONFINITE.
 *
 * First iterate of a step: the last iterate of the previous step (all four
 * components); after oci_setup or oci_set_state it is psi_prev copied to both
 * time levels.  After a step the state psi_{k-1/2} <- psi_{k+1/2} (the time
 * update).
 *
 * Precision:
 *   OCI_FP64          cell systems factored (LU, partial pivoting) and applied
 *                     in FP64.
 *   OCI_FP32_REFINED  factored and applied in FP32; each iteration is the
 *                     refinement step Psi^(l+1) = Psi^(l) + A^-1 (b - A Psi^(l))
 *                     with the residual in FP64 (power-of-two scaled before the
 *                     FP32 solve).  Its fixed point is the FP64 one; the norm
 *                     and the time update stay FP64.
 *
 * Memory and streams:
 *   Pointers named *_dev are device memory owned by the caller; host arrays are
 *   read during the call only.  All arrays are C order, float64.  The library
 *   allocates no device memory: everything it keeps (factors, iterates,
 *   control blocks) lives in the caller's workspace, sized by
 *   oci_workspace_bytes and aligned to 256 bytes.  All GPU work is enqueued on
 *   the stream given to oci_setup (a hipStream_t passed as void *; NULL = the
 *   null stream).  oci_setup synchronises that stream once (to report a
 *   singular cell); oci_step and si_step may synchronise it to learn
 *   convergence but never the device.  Step results land in *info_dev
 *   asynchronously.  A handle is not thread-safe; one handle must not be used
 *   from two streams at once.
 *
 * Co-residency: the iteration loop of a step is one persistent launch whose
 *   workgroups wait on each other (edge hand-offs, partial sums, barriers).
 *   The launch is sized so that all its workgroups fit on the device at once,
 *   which holds only while nothing else occupies the compute units: a step
 *   must not overlap other kernels on the same device (another handle's step
 *   on a second stream, other work of the caller, another process).  Every
 *   wait is bounded; if a workgroup could not be scheduled the waits expire,
 *   the step stops and its info reports OCI_ERR_DEVICE.  A step never hangs.
 *
 * Errors: every call returns an oci_status; negative values are errors and
 * leave the handle usable unless stated.  Arguments are validated on the host
 * before anything is launched.
 */
#ifndef OCI_H
#define OCI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OCI_OK = 0,
    OCI_NOT_CONVERGED = 1,     /* max_iters reached (step result, in info) */
    OCI_NONFINITE = 2,         /* e_l not finite (step result, in info) */
    OCI_ERR_INVALID = -1,      /* bad argument; nothing was launched */
    OCI_ERR_HIP = -2,          /* a HIP runtime call failed */
    OCI_ERR_SINGULAR = -3,     /* a cell matrix has a zero pivot */
    OCI_ERR_WORKSPACE = -4,    /* workspace NULL, too small or misaligned */
    OCI_ERR_UNSUPPORTED = -5,  /* shape or option beyond the compiled kernels (4NG > 512;
                                  the structured solve with FP32, the angular norm or
                                  G > 8; red-black or periodic without it) */
    OCI_ERR_DEVICE = -6,       /* a device-side wait expired (a workgroup of the
                                  persistent launch was not co-resident) */
    OCI_ERR_TOO_LARGE = -7     /* oci_setup_static: the workspace would exceed its
                                  64 MiB static array */
} oci_status;

typedef enum { OCI_FP64 = 0, OCI_FP32_REFINED = 1 } oci_precision;
typedef enum { OCI_NORM_SCALAR = 0, OCI_NORM_ANGULAR = 1 } oci_norm;

/* How a cell system is solved in each OCI iteration.
 *   OCI_SOLVE_DENSE       the factored (4NG)^2 matrix, kept as its inverse
 *                         (the paper's stored-LHS design, section 2.5).
 *   OCI_SOLVE_STRUCTURED  the same exact solve through the structure of A_j
 *                         (section 2.4: block diagonal 4x4 corner blocks minus
 *                         a scattering coupling of rank 4G): the corner blocks
 *                         are inverted in closed form and the coupling through
 *                         a 4G x 4G capacitance matrix inverted once per cell
 *                         at setup.  FP64 only (precision OCI_FP64), scalar
 *                         norm only, G <= 8; no n x n factors are stored.  SI
 *                         is available on the same handle. */
typedef enum { OCI_SOLVE_DENSE = 0, OCI_SOLVE_STRUCTURED = 1 } oci_solver;

/* Order in which the cells of one OCI iteration are solved.
 *   OCI_ORDER_JACOBI     every cell from the previous iterate (cell-wise block
 *                        Jacobi, eq. oci; the paper's OCI).
 *   OCI_ORDER_RED_BLACK  the even cells from the previous iterate, then the
 *                        odd cells from the even cells' new values (the block
 *                        Gauss-Seidel ordering the paper's introduction names
 *                        as the alternative); the same fixed point, the
 *                        iteration operator's spectral radius squared.  One
 *                        iteration still solves every cell once.  Structured
 *                        solve only. */
typedef enum { OCI_ORDER_JACOBI = 0, OCI_ORDER_RED_BLACK = 1 } oci_ordering;

/* Boundary of the slab.
 *   OCI_BOUNDARY_INCIDENT  prescribed incident fluxes (vacuum when NULL).
 *   OCI_BOUNDARY_PERIODIC  a periodic mesh: cell 0 and cell J - 1 are
 *                          neighbours (the setting of the paper's Fourier
 *                          analysis, section 2.3, and of its verification
 *                          runs); incident-flux arguments are ignored.
 *                          Structured solve only. */
typedef enum { OCI_BOUNDARY_INCIDENT = 0, OCI_BOUNDARY_PERIODIC = 1 } oci_boundary;

/* Problem description.  Host pointers, read during oci_setup only. */
typedef struct {
    int32_t J;                /* cells, >= 1 */
    int32_t N;                /* Gauss-Legendre angles, even, >= 2 */
    int32_t G;                /* energy groups, >= 1; 4 N G <= 512 */
    const double *dx;         /* [J] cell widths (cm), > 0 */
    const double *sigma_t;    /* [J][G] total cross sections (1/cm), >= 0 */
    const double *sigma_s;    /* [J][G][G], [j][g][gp] = scattering gp -> g, >= 0 */
    const double *speed;      /* [G] particle speeds (cm/s), > 0 */
    double dt;                /* time-step size (s), > 0 */
    double tol;               /* epsilon of the stopping rule, >= 0 */
    int32_t max_iters;        /* >= 1 */
    int32_t fixed_iters;      /* > 0: run exactly this many iterations per step
                                 with no stopping test (lock-step comparisons) */
    int32_t precision;        /* oci_precision */
    int32_t norm;             /* oci_norm, OCI only */
    int32_t solver;           /* oci_solver (0 = dense) */
    int32_t ordering;         /* oci_ordering (0 = Jacobi) */
    int32_t boundary;         /* oci_boundary (0 = incident fluxes) */
} oci_desc;

/* Per-step result, written to device memory by oci_step / si_step. */
typedef struct {
    int32_t iterations;       /* iterations performed in the step */
    int32_t status;           /* OCI_OK, OCI_NOT_CONVERGED or OCI_NONFINITE */
    double e_last;            /* e_l of the last iteration */
    double rho_e;             /* e_l / e_{l-1} of the last iteration (NaN if l = 0) */
} oci_step_info;

typedef struct oci_handle oci_handle;

/* Bytes of device workspace oci_setup needs for this description (OCI and SI
 * together).  Returns OCI_ERR_INVALID / OCI_ERR_UNSUPPORTED for a bad one. */
int oci_workspace_bytes(const oci_desc *desc, size_t *bytes);

/* Validate, build the quadrature, upload the material data into the
 * workspace, then assemble every cell matrix A_j (eqs. Aj, scatter_mg,
 * fullOCIlhs) on the device and factor it (LU with partial pivoting, the
 * paper's gesv factorisation) in the requested precision; the factors are
 * kept, as the inverse they define, for every iteration of every step.  Also
 * prepares the 4x4 SI cell systems.  State psi_prev = 0.  Synchronises the
 * stream.  On success *out receives a handle (host memory, owned by the
 * caller until oci_destroy). */
int oci_setup(const oci_desc *desc, void *workspace_dev, size_t workspace_bytes,
              void *stream, oci_handle **out);

/* oci_setup without a caller-provided workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  The workspace is a 64 MiB array in the
 * library's device memory, one per device, held from the library's load on
 * that device until the process ends; this call allocates no device memory
 * and calls no allocating routine.  A problem whose oci_workspace_bytes
 * exceeds 64 MiB is rejected with OCI_ERR_TOO_LARGE before anything runs.
 * Every handle this call returns on one device shares that device's array
 * and the array keeps the last call's contents (the setup clears what a step
 * needs to start from zero): a new oci_setup_static on the device takes the
 * array over, so only the handle it returns may be used afterwards, and calls
 * on two handles of one device that overlap in time race.  Otherwise the
 * handle behaves as one from oci_setup (same kernels, same results). */
int oci_setup_static(const oci_desc *desc, void *stream, oci_handle **out);

/* Replace the state psi_{k-1/2}: psi_prev_dev [J][G][N][2] (L, R corners),
 * NULL = zero.  The first iterate of the next step becomes psi_prev copied to
 * both time levels.  Asynchronous device-to-device copy. */
int oci_set_state(oci_handle *h, const double *psi_prev_dev);

/* Copy the state psi_{k-1/2} into psi_prev_dev [J][G][N][2]. Asynchronous. */
int oci_get_state(const oci_handle *h, double *psi_prev_dev);

/* Checkpoint for a bit-for-bit restart: everything a later step depends on
 * besides the problem itself, psi_{k-1/2} [J][G][N][2] and the first iterate
 * of the next step [J][G][N][4] (the last iterate of the previous step, or
 * psi_prev on both time levels after oci_setup / oci_set_state; reading R3 of
 * section 2.1's iteration).  oci_get_checkpoint copies both out;
 * oci_set_checkpoint loads them into a handle set up from the same
 * description, whose later steps then equal, bit for bit, those of the handle
 * the checkpoint came from.  Asynchronous device-to-device copies on the
 * handle's stream; all pointers device memory owned by the caller. */
int oci_get_checkpoint(const oci_handle *h, double *psi_prev_dev, double *psi_iter_dev);
int oci_set_checkpoint(oci_handle *h, const double *psi_prev_dev, const double *psi_iter_dev);

/* One OCI time step (Algorithm 2; eq. oci).
 *   q_dev         [J][G][4] isotropic source Q at (k,L), (k,R), (k+1/2,L),
 *                 (k+1/2,R); NULL = no source
 *   inc_left_dev  [2][G][N/2] incident flux at x = 0 for the mu > 0 angles in
 *                 ascending order, time level k then k+1/2; NULL = vacuum
 *   inc_right_dev [2][G][N/2] the same at x = X for the mu < 0 angles
 *   phi_out_dev   [J][G][4] scalar flux of the last iterate (required)
 *   psi_out_dev   [J][G][N][4] angular flux of the last iterate, NULL = skip
 *   info_dev      one oci_step_info in device memory (required)
 * The inputs must stay valid until the stream reaches the end of the step. */
int oci_step(oci_handle *h, const double *q_dev, const double *inc_left_dev,
             const double *inc_right_dev, double *phi_out_dev, double *psi_out_dev,
             oci_step_info *info_dev);

/* nsteps consecutive OCI time steps (Algorithm 2 repeated over the steps
 * of section 2.1's time discretisation); the same result, step for step, as
 * nsteps calls of oci_step with each step's sources.
 *   q_dev, q_stride      step k's Q is q_dev + k q_stride ([J][G][4] each;
 *                        q_stride = 0: the same Q every step, as in the test
 *                        problem of the paper's GPU performance study,
 *                        section 3.2, table rosa_test); q_dev NULL = none
 *   inc_left_dev, inc_right_dev, inc_stride
 *                        step k's incident fluxes are inc_*_dev + k inc_stride
 *                        ([2][G][N/2] each; 0: the same every step); NULL =
 *                        vacuum
 *   phi_out_dev          [nsteps][J][G][4] scalar flux of each step's last
 *                        iterate
 *   psi_out_dev          [J][G][N][4] angular flux of the last step's last
 *                        iterate, NULL = skip
 *   info_dev             nsteps oci_step_info records in device memory
 * With the register-resident kernel (see oci_get_config) the steps run in one
 * launch: each step's stop turns the iterate over to the next step inside the
 * kernel, so the inverse rows are loaded once for all of them.  Otherwise it
 * calls oci_step nsteps times.  OCI_ERR_INVALID if nsteps < 1, a stride is
 * negative or an output is NULL. */
int oci_run_steps(oci_handle *h, int32_t nsteps, const double *q_dev, int64_t q_stride,
                  const double *inc_left_dev, const double *inc_right_dev, int64_t inc_stride,
                  double *phi_out_dev, double *psi_out_dev, oci_step_info *info_dev);

/* Capture n_steps OCI time steps into a HIP graph held by the handle (its
 * stream must not be NULL), with per-step arguments for time-dependent
 * sources Q_k, Q_{k+1/2} and incident fluxes psi_inc(t) (section 2.1):
 * host arrays of n_steps device pointers (q_dev, inc_left_dev, inc_right_dev,
 * psi_out_dev: arrays or entries may be NULL, as in oci_step; phi_out_dev:
 * every entry required) and info_dev, n_steps oci_step_info in device
 * memory.  Nothing runs until oci_replay_steps.  The steps' kernels are those
 * of oci_step; the first iterate of each step is decided on the device (the
 * state after oci_set_state, else the last iterate), so a replay equals
 * n_steps oci_step calls bit for bit.  A new capture replaces the graph;
 * oci_destroy releases it. */
int oci_capture_steps(oci_handle *h, int32_t n_steps, const double *const *q_dev,
                      const double *const *inc_left_dev, const double *const *inc_right_dev,
                      double *const *phi_out_dev, double *const *psi_out_dev, oci_step_info *info_dev);

/* Launch the captured steps on the handle's stream (asynchronous);
 * OCI_ERR_INVALID if nothing was captured. */
int oci_replay_steps(oci_handle *h);

/* One source-iteration time step (Appendix A, Algorithm 1) on the same state
 * and with the same arguments as oci_step. */
int si_step(oci_handle *h, const double *q_dev, const double *inc_left_dev,
            const double *inc_right_dev, double *phi_out_dev, double *psi_out_dev,
            oci_step_info *info_dev);

/* Instrumentation (not part of the method).  With on != 0, every later
 * oci_step / si_step records a pair of HIP events on the handle's stream
 * around its iteration kernels (OCI: the one persistent launch; SI: all sweep
 * and flux launches of the step).  Event pairs are host-side objects owned by
 * the handle; enabling costs two event records per step. */
int oci_profile_enable(oci_handle *h, int on);

/* Synchronise on the recorded events and return, since the last read (or
 * the enable), the summed milliseconds of the iteration kernels in *ms and
 * the number of steps recorded in *steps; then forget them. */
int oci_profile_read(oci_handle *h, double *ms, int32_t *steps);

/* Autotuner: time the candidate launch shapes of the persistent OCI kernel
 * on this handle's own problem and keep the fastest.  Candidates: 256 or
 * 1024 threads per workgroup (4 or 16 cells per tile at n <= 64), the
 * workgroup-local kernel with register-resident or streamed inverse rows or
 * the global-memory kernel, and barrier arrival groups of 16 or 64
 * workgroups.  Each runs `iters` iterations of one step from the zero state
 * (no stopping test), timed with HIP events.  Synchronises the stream; the
 * state is zero afterwards (call it right after oci_setup).  config, if not
 * NULL, receives the chosen shape as oci_get_config reports it. */
int oci_autotune(oci_handle *h, int32_t iters, int32_t *config);

/* Per-iteration record of the stopping quantity (instrumentation for the
 * convergence studies of section 3.1): with e_hist_dev non-NULL, every later
 * OCI step writes e_l of its iteration l (l = 1, 2, ...) into
 * e_hist_dev[l - 1] for l <= capacity (device memory, owned by the caller;
 * entries beyond the step's iteration count keep their old contents; a
 * multi-step launch leaves the last step's record).  NULL turns it off. */
int oci_set_history(oci_handle *h, double *e_hist_dev, int32_t capacity);

/* Current launch shape: config[6] = {threads per workgroup, local kernel (0/1;
 * for the structured solve: tile inputs staged in LDS ahead of the arithmetic),
 * register-resident rows (0/1), barrier group size, workgroups, tiles}. */
int oci_get_config(const oci_handle *h, int32_t *config);

/* Release the host-side handle.  The workspace stays the caller's. */
int oci_destroy(oci_handle *h);

/* ---------------------------------------------------------------- batches
 * Many independent slab problems (uneven J, N, G; one precision) advanced
 * together: every batched time step runs one persistent launch in which slab
 * k is served by its own block of workgroups (sized in proportion to its
 * factor bytes per iteration, J x (4NG)^2), with its own control block,
 * barrier and stopping decision, so slabs converge independently.  The
 * iteration of each slab is the same OCI iteration as oci_step (eq. oci,
 * Algorithm 2), through the factors kept in global memory.  Steps can be
 * captured once into a HIP graph and replayed. */
typedef struct oci_batch oci_batch;

/* Workspace bytes for nslab descriptions (all of one precision). */
int oci_batch_workspace_bytes(int32_t nslab, const oci_desc *descs, size_t *bytes);

/* Set up every slab (as oci_setup, each in its own part of the workspace)
 * and lay out the batched launch.  Synchronises the stream.  Returns
 * OCI_ERR_UNSUPPORTED when the slabs cannot all be given a co-resident
 * workgroup. */
int oci_batch_setup(int32_t nslab, const oci_desc *descs, void *workspace_dev,
                    size_t workspace_bytes, void *stream, oci_batch **out);

/* Bind the per-slab step arguments used by every later oci_batch_step and
 * by a captured graph: host arrays of nslab device pointers (q, incident
 * fluxes: entries or whole arrays may be NULL, as in oci_step; phi_out:
 * required) and info_dev, nslab oci_step_info in device memory.  Uploads the
 * launch table and synchronises the stream. */
int oci_batch_bind(oci_batch *b, const double *const *q_dev, const double *const *inc_left_dev,
                   const double *const *inc_right_dev, double *const *phi_out_dev,
                   oci_step_info *info_dev);

/* Bind n_steps argument sets (1 <= n_steps <= 64), one per time step, for
 * time-dependent sources and incident fluxes (the Q_k, Q_{k+1/2} and
 * psi_inc(t) of section 2.1): host arrays of n_steps x nslab device pointers,
 * entry [i][k] for step i of slab k (q, incident fluxes: entries or whole
 * arrays may be NULL; phi_out: every entry required), and info_dev,
 * n_steps x nslab oci_step_info in device memory.  Eager steps use the sets
 * in order, cyclically; a capture of n steps records the next n sets.
 * oci_batch_bind is the one-set case.  Discards a captured graph, uploads
 * the launch tables and synchronises the stream. */
int oci_batch_bind_steps(oci_batch *b, int32_t n_steps, const double *const *q_dev,
                         const double *const *inc_left_dev, const double *const *inc_right_dev,
                         double *const *phi_out_dev, oci_step_info *info_dev);

/* One time step of every slab with the next bound argument set
 * (asynchronous; results in that set's outputs). */
int oci_batch_step(oci_batch *b);

/* Capture n_steps batched steps into a HIP graph held by the batch (needs a
 * non-null stream) and instantiate it; nothing runs until the first
 * oci_batch_replay.  Step i of the graph uses the bound argument set
 * (next + i) mod n_bound, next being the set the next eager step would use.
 * Each replay runs the n_steps steps from the current state. */
int oci_batch_capture(oci_batch *b, int32_t n_steps);
int oci_batch_replay(oci_batch *b);

/* State of slab k, as oci_set_state / oci_get_state. */
int oci_batch_set_state(oci_batch *b, int32_t k, const double *psi_prev_dev);
int oci_batch_get_state(const oci_batch *b, int32_t k, double *psi_prev_dev);

/* Batch autotuning: re-size every slab's block of workgroups from the
 * iterations of the last step enqueued (read from its argument set's info
 * records): a slab's time is modelled as iterations x (tiles per workgroup x
 * cost of a tile + one grid barrier), and the blocks are chosen to minimise
 * the largest slab time within the co-resident capacity, so slabs that
 * converge slowly get more of the launch.  Before any rebalance the blocks
 * follow the tile counts alone.  OCI_ERR_INVALID before any step.
 * Synchronises the stream; a captured graph is discarded (capture again
 * afterwards). */
int oci_batch_rebalance(oci_batch *b);

/* Launch geometry: total workgroups and, if nwg_per_slab is not NULL, the
 * workgroups of each slab ([nslab]). */
int oci_batch_info(const oci_batch *b, int32_t *nwg_total, int32_t *nwg_per_slab);

/* Release the batch and its slab handles (the workspace stays the caller's). */
int oci_batch_destroy(oci_batch *b);

/* Static text for a status code. */
const char *oci_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* OCI_H */
