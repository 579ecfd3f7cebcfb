/*
 * cmcg.h -- C ABI of the MI355X (gfx950) controllability-CG solver for
 * time-harmonic Maxwell's equations.
 *
 * Method (Chaumont-Frelet, Grote, Lanteri, Tang, "A controllability method
 * for Maxwell's equations"):
 *   Problem (Section 1, eq. (1.1)): find complex fields e, h with
 *       i omega eps e + sigma e + curl h = j,   i omega mu h - curl e = 0,
 *   e x n = 0 on the PEC boundary, an impedance (Silver-Mueller) condition
 *   with data g on the rest.  The time-domain problem eq. (1.2) is driven by
 *   Re(j e^{i omega t}); CMCG (Section 2.2, Algorithms 1-3) searches the
 *   initial state U0 with P_psi U0 = U0 over one period T = 2 pi / omega by
 *   conjugate gradients on J(U0) = 1/2 ||(I - P) U0 - G||^2_{eps,mu}, where
 *   every gradient costs one forward and one backward (adjoint, P* = S P S)
 *   period of an explicit upwind DG / Runge-Kutta scheme (Sections 5.2.2 and 5.3),
 *   and returns the filtered field F_psi U0 = (2/T) int_0^T U(t) e^{-i w t}
 *   dt, computed on the fly during a last forward period (Section 5.4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Arrays are row-major and contiguous.  Indices are int64.
 *  - Element map: x = v0 + xi1 (v1 - v0) + xi2 (v2 - v0) + xi3 (v3 - v0) on
 *    the reference tetrahedron {xi >= 0, xi1 + xi2 + xi3 <= 1}; v0..v3 are
 *    the element's vertices in the order given in tet[K][4].  Both
 *    orientations are accepted.
 *  - Local face f is opposite local vertex f.
 *  - DG nodes of P_q (q = 1, 2, 3): xi = (i, j, k) / q with i + j + k <= q,
 *    ordered with k slowest, then j, then i fastest.  Np = (q+1)(q+2)(q+3)/6
 *    nodes per element, Nfp = (q+1)(q+2)/2 per face.  The nodes of face f are
 *    the element nodes lying on it, in element node order.
 *  - "Field" arrays at nodes: [K][Np][3] (x, y, z components).
 *  - "Dof vectors" (debug entry points): [K][6][Np], components
 *    (Ex, Ey, Ez, Hx, Hy, Hz) -- the library's internal layout.
 *  - Time dependence e^{+i omega t}; field sign convention of eq. (1.2).
 *  - Impedance faces use the dissipative Silver-Mueller condition
 *    E x n - Z H_tau = G with Z = sqrt(mu/eps) of the adjacent element.
 *
 * Errors: every int-returning function returns CMCG_OK (0) on success,
 * CMCG_NOT_CONVERGED (1) when a solve stopped at max_iter (its result is
 * valid and flagged), or a negative CMCG_ERR_* code; cmcg_last_error()
 * then describes the failure (thread-local).  No exception crosses the ABI.
 * Handles are owned by the caller once returned and released with the
 * matching *_destroy (NULL is accepted).  Input arrays are copied; the
 * caller may free them after return.  A handle must not be used from two
 * threads at once.
 *
 * Device: objects live on the HIP device that is current when they are
 * created; later calls must be made with that device current.
 */
#ifndef CMCG_H
#define CMCG_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CMCG_OK = 0,
    CMCG_NOT_CONVERGED = 1,
    CMCG_ERR_ARG = -1,       /* invalid argument (NULL, size, range)          */
    CMCG_ERR_MESH = -2,      /* degenerate / non-conforming / untagged mesh    */
    CMCG_ERR_NOMEM = -3,     /* device memory exhausted or over budget         */
    CMCG_ERR_DEVICE = -4,    /* a HIP runtime call failed                      */
    CMCG_ERR_UNSTABLE = -5,  /* non-finite values appeared (step too large)    */
    CMCG_ERR_BREAKDOWN = -6, /* CG breakdown: (D, A) <= 0 or not finite        */
    CMCG_ERR_STATE = -7,     /* call not valid in the object's current state   */
    CMCG_ERR_TOO_LARGE = -8  /* serving: the request's footprint exceeds the
                                engine's whole budget (never admissible)        */
};

enum { CMCG_FP64 = 0, CMCG_FP32 = 1 };                   /* field precision  */
enum { CMCG_TAG_INTERIOR = 0, CMCG_TAG_PEC = 1, CMCG_TAG_IMPEDANCE = 2 };
enum { CMCG_SCHEME_AUTO = 0, CMCG_SCHEME_RK2 = 2, CMCG_SCHEME_RK4 = 4 };
enum { CMCG_FLUX_UPWIND = 0, CMCG_FLUX_CENTRED = 1 };

typedef struct cmcg_mesh cmcg_mesh;
typedef struct cmcg_space cmcg_space;
typedef struct cmcg_problem cmcg_problem;
typedef struct cmcg_result cmcg_result;

/* Solver options (Algorithm 3 and the time discretisation of Section 5.3). */
typedef struct cmcg_options {
    double tol;          /* stop when ||R_l|| <= tol ||R_0|| in the eps,mu norm */
    int max_iter;        /* CG iteration cap (Algorithm 3's l_max)             */
    int fixed_iters;     /* > 0: run exactly this many CG iterations, ignoring
                            tol (parity testing at a fixed iteration count)     */
    double cfl;          /* c_q of the CFL rule dt <= c_q min sqrt(mu eps) rho;
                            <= 0 selects 0.20 / 0.16 / 0.12 for q = 1 / 2 / 3   */
    int steps;           /* > 0: force M steps per period instead of the CFL M */
    int scheme;          /* CMCG_SCHEME_*: AUTO = RK2 for q = 1, RK4 otherwise;
                            RK2 pairs with the trapezoid filter, RK4 with the
                            cubic-Hermite filter                                */
    int flux;            /* CMCG_FLUX_UPWIND (the paper's) or _CENTRED (tests);
                            impedance faces are always upwind                   */
    int use_graph;       /* 1: replay each period from a captured hipGraph      */
    int residual_refresh;/* > 0: every this many iterations replace R by the
                            true gradient (costs two periods); <= 0 = never.
                            FP32 fields keep the state compensated (FP32 +
                            bfloat16 low part), which holds the rounding floor
                            of the residual near 2e-7 on the 48000-tet P3
                            problem, so the recursive residual needs no
                            refresh at the usual tolerances                    */
    /* Optional progress report, called on the host after every CG iteration
     * with the iteration count and ||R_l|| / ||R_0||; a non-zero return value
     * stops the iteration (the result is then flagged NOT_CONVERGED).  NULL =
     * no report. */
    int (*progress)(void* ctx, int iter, double rel_res);
    void* progress_ctx;
    /* Run-up (Section 6 mentions it as a way to accelerate CMCG): > 0 runs
     * that many limiting-amplitude periods U <- P_psi U (time stepping with the
     * source) from the initial guess before Algorithm 3 starts, which then
     * starts from their end state; the periods count in stats.periods.  0 =
     * none (the paper's zero initialisation); < 0 is CMCG_ERR_ARG. */
    int runup;
    /* 1: before its first period the solve picks the stage-kernel variant with
     * the autotuner (cmcg_autotune_stage; batched solves time the batched
     * launch), once per (device, q, precision, K, members) in the process,
     * and keeps it as the process-wide choice for (q, precision).  The
     * serving engine ignores it (slots run concurrently; tune beforehand).
     * 0 = keep the current choice. */
    int autotune;
    /* Local time stepping for locally refined meshes (the paper's concluding
     * remarks), 2..64: every period is M coarse steps of H = T / M, where M is
     * the smallest count with H / lts_ratio no longer than the smallest
     * element's CFL step (o->steps forces M); elements whose own CFL step
     * c_q sqrt(mu eps) rho is shorter than H are fine and take lts_ratio
     * substeps of the base scheme (RK2 / RK4) per coarse step, the others
     * enter through the Taylor polynomial of the solution at the coarse step's
     * start (Runge-Kutta-based local time stepping).  Backward periods are
     * the exact adjoint of that propagator, so CMCG's gradient stays exact.
     * Fields stay in the space's precision without the compensated FP32
     * state; periods run without graph capture.  Tetrahedral spaces, single
     * frequency; not accepted by cmcg_solve_batch.  0 or 1 = global steps. */
    int lts_ratio;
} cmcg_options;

/* Fills *o with defaults: tol 1e-8, max_iter 1000, fixed_iters 0, cfl 0,
 * steps 0, scheme AUTO, flux UPWIND, use_graph 1, residual_refresh 0,
 * progress NULL, runup 0, autotune 0, lts_ratio 0. */
void cmcg_options_default(cmcg_options* o);

/* Solve statistics. */
typedef struct cmcg_stats {
    int iters;           /* CG iterations performed                            */
    int periods;         /* periods simulated (2 per iteration + init + filter) */
    int steps;           /* M, time steps per period                            */
    int status;          /* CMCG_OK or CMCG_NOT_CONVERGED                       */
    double dt;           /* T / M                                               */
    double rel_res;      /* final ||R_l|| / ||R_0||                             */
    double J0;           /* J(U0^(0)) = 1/2 ||G||^2 for a zero initial guess     */
    double seconds;      /* wall time of the solve (inputs resident on device)  */
    double seconds_to_1e6; /* wall time until ||R||/||R0|| <= 1e-6 (-1: never)  */
    double dof_updates;  /* 6 Np K x steps executed over all periods            */
    double res0;         /* ||R_0|| in the eps,mu norm: the first residual, the
                            scale of the stop rule (0 for the FW iteration)     */
} cmcg_stats;

const char* cmcg_last_error(void);
const char* cmcg_version(void);

/* ---------------------------------------------------------------- mesh -- */
/* Conforming tetrahedral mesh (Section 5.2.2: conforming simplicial mesh; each
 * boundary face lies entirely on the PEC or the impedance part).
 *   xyz[nv][3]   vertex coordinates
 *   tet[K][4]    vertex indices (0-based)
 *   face_tag     [K][4] (local face f opposite local vertex f): for boundary
 *                faces CMCG_TAG_PEC or CMCG_TAG_IMPEDANCE; ignored on interior
 *                faces.  NULL tags every boundary face impedance.
 * Errors: CMCG_ERR_ARG (NULL, nv < 4, K < 1, K >= 2^26 -- the neighbour
 * index shares a 32-bit connectivity word with the face and permutation
 * codes --, index out of range), CMCG_ERR_MESH (zero volume, a face shared by
 * more than two elements, an untagged boundary face). */
/* Element order for locality (host only, no device work): order[K] receives
 * a permutation of 0..K-1 that sorts the element centroids along a Morton
 * (Z-order) curve over their bounding cube, 21 bits per axis, ties kept in
 * input order.  The stage kernels process elements in blocks of consecutive
 * indices and read face neighbours through the caches, so a mesh whose
 * elements are numbered without spatial locality runs slower (a randomly
 * numbered 384000-tet cube: +15% P3, +17% P2 per stage); creating the mesh
 * from tet[order[i]] (with face_tag[order[i]] and every per-element input
 * permuted alike) restores the locality.  The library never reorders
 * elements itself: its arrays keep the caller's element order.
 * Errors: CMCG_ERR_ARG (NULL, nv < 1, K < 1, index out of range, non-finite
 * coordinates). */
int cmcg_mesh_locality_order(int64_t nv, const double* xyz, int64_t K, const int64_t* tet, int64_t* order);

int cmcg_mesh_create(int64_t nv, const double* xyz, int64_t K, const int64_t* tet,
                     const int8_t* face_tag, cmcg_mesh** out);
/* Conforming triangle mesh of the 2-D transverse-magnetic setting (Section
 * 5.1: fields independent of the third coordinate, e = E_3 and h = (H_1,
 * H_2); Section 5.2.2: its DG scheme on triangles, edge sets interior / PEC /
 * impedance).
 *   xy[nv][2]     vertex coordinates
 *   tri[K][3]     vertex indices (0-based), either orientation
 *   edge_tag      [K][3] (local edge f opposite local vertex f): for boundary
 *                 edges CMCG_TAG_PEC or CMCG_TAG_IMPEDANCE; NULL tags every
 *                 boundary edge impedance.
 * Spaces on such a mesh hold (e, h1, h2): dof vectors [K][3][Np] with Np =
 * (q+1)(q+2)/2 equispaced nodes (i, j)/q, j slowest; the CFL constants
 * default to the paper's c_1 = 0.24 and c_3 = 0.12 (c_2 = 0.16) with rho_K
 * the diameter of the inscribed circle.  Layouts of the other calls on 2-D
 * spaces: cmcg_space_nodes xy[K][Np][2]; problem current j[K][Np] (the e
 * component; device form alike), impedance data g[K][3][Nfp] (the scalar G of
 * e + Z h x n = G, h x n = h1 n2 - h2 n1, edge nodes from the edge's
 * lower-numbered vertex); cmcg_result_fields e[K][Np], h[K][Np][2].  2-D
 * problems are solved by cmcg_solve, cmcg_fw_solve, cmcg_solve_batch and the
 * serving engine; cmcg_problem_create_harmonics takes j[nh][K][Np] on a 2-D
 * space; the stage autotuner returns CMCG_ERR_ARG for them.
 * Errors: CMCG_ERR_ARG (NULL, nv < 3, K < 1, K >= 2^26, index out of range),
 * CMCG_ERR_MESH (zero area, an edge shared by more than two triangles, an
 * untagged boundary edge). */
int cmcg_mesh2d_create(int64_t nv, const double* xy, int64_t K, const int64_t* tri,
                       const int8_t* edge_tag, cmcg_mesh** out);
/* Dimension of a mesh: 3 (tetrahedra) or 2 (triangles). */
int cmcg_mesh_dim(const cmcg_mesh* m, int* dim);
void cmcg_mesh_destroy(cmcg_mesh* m);
int cmcg_mesh_info(const cmcg_mesh* m, int64_t* K, int64_t* n_boundary_faces,
                   double* min_rho);

/* --------------------------------------------------------------- space -- */
/* Broken nodal space P_q(T_h)^6 on the mesh (Section 5.2.2), field precision
 * CMCG_FP64 or CMCG_FP32 (time stepping in that precision; CG vectors,
 * inner products, alpha/beta and the filter accumulator always FP64).
 * Uploads geometry and connectivity to the current device.  The mesh may be
 * destroyed afterwards. */
int cmcg_space_create(const cmcg_mesh* m, int q, int precision, cmcg_space** out);
void cmcg_space_destroy(cmcg_space* s);
int cmcg_space_info(const cmcg_space* s, int* q, int* Np, int* Nfp, int64_t* K,
                    int64_t* ndof);
/* Physical coordinates of the DG nodes, xyz[K][Np][3] (host). */
int cmcg_space_nodes(const cmcg_space* s, double* xyz);

/* ------------------------------------------------------------- problem -- */
/* Problem data (Section 1, eq. (1.1)):
 *   eps[K], mu[K] > 0, sigma[K] >= 0 (NULL = 0): piecewise constant;
 *   omega > 0;
 *   j_re / j_im [K][Np][3]: nodal coefficients of j in the DG space (j_im
 *   may be NULL = 0);
 *   g_re / g_im [K][4][Nfp][3]: impedance boundary data at face nodes (read on
 *   impedance faces only; NULL = 0).
 * Host pointers.  The space may be destroyed afterwards. */
int cmcg_problem_create(const cmcg_space* s, const double* eps, const double* mu,
                        const double* sigma, double omega, const double* j_re,
                        const double* j_im, const double* g_re, const double* g_im,
                        cmcg_problem** out);
/* Same, with j_re / j_im ([K][Np][3]) and g_re / g_im ([K][4][Nfp][3];
 * 2-D spaces: j [K][Np], g [K][3][Nfp]) resident in device memory; each may
 * be NULL (= 0).  Read in order on `stream`, which is synchronised before
 * return; the caller may free them afterwards.  eps, mu, sigma are host
 * arrays.  Errors as cmcg_problem_create, CMCG_ERR_DEVICE when a copy
 * fails. */
int cmcg_problem_create_device(const cmcg_space* s, const double* eps, const double* mu,
                               const double* sigma, double omega, const double* j_re_dev,
                               const double* j_im_dev, const double* g_re_dev,
                               const double* g_im_dev, hipStream_t stream, cmcg_problem** out);
/* Several frequencies in one solve (the paper's concluding remarks): a
 * current made of nh (1..8) harmonics of a base angular frequency omega0,
 * J(t) = sum_h Re(j_h e^{i k[h] omega0 t}) with distinct integers k[h] >= 1,
 * is periodic with T = 2 pi / omega0; cmcg_solve / cmcg_fw_solve then solve
 * over that period and filter every harmonic at its own frequency k[h]
 * omega0 (Section 5.4 weights), so one solve yields nh time-harmonic fields
 * (cmcg_result_filtered_harmonic_device).  The time step follows the CFL rule
 * for the period T; its accuracy at the highest harmonic is the caller's
 * choice (o->steps forces M).  j_re / j_im: [nh][K][Np][3] host arrays
 * (j_im may be NULL); no boundary data.  CMCG_ERR_ARG for nh out of range or
 * repeated / non-positive k.  Not accepted by cmcg_solve_batch. */
int cmcg_problem_create_harmonics(const cmcg_space* s, const double* eps, const double* mu,
                                  const double* sigma, double omega0, int nh, const int* k,
                                  const double* j_re, const double* j_im, cmcg_problem** out);
void cmcg_problem_destroy(cmcg_problem* p);
/* Time steps per period M and dt = T / M that `o` selects for this problem
 * (CFL rule of Section 5.3; with o->lts_ratio > 1 the coarse steps). */
int cmcg_problem_steps(const cmcg_problem* p, const cmcg_options* o, int* M, double* dt);
/* Elements that local time stepping with `o` (o->lts_ratio > 1) treats as
 * fine; fine[K] (host, nullable) receives 1 / 0 per element, *n_fine the
 * count.  CMCG_ERR_ARG when o asks for no local time stepping. */
int cmcg_problem_lts_fine(const cmcg_problem* p, const cmcg_options* o, int8_t* fine, int64_t* n_fine);

/* ---------------------------------------------------------------- solve -- */
/* Algorithm 3 from the zero initial guess (or `u0_dev`, a device dof vector
 * [K][6][Np] FP64, when not NULL), then the filter period.  Work is ordered
 * on `stream` (NULL = the default stream); the call returns when the result
 * is complete.  Returns CMCG_OK, CMCG_NOT_CONVERGED (result valid), or an
 * error (no result).  When the recursive residual grows past 100 times the
 * smallest value it has reached (the rounding floor of FP32 fields lies above
 * the tolerance), the iteration stops, the filter runs on the best iterate,
 * and the status is CMCG_NOT_CONVERGED with rel_res the best value. */
int cmcg_solve(cmcg_problem* p, const cmcg_options* o, const double* u0_dev,
               hipStream_t stream, cmcg_result** out);

/* Limiting-amplitude ("full wave", FW) iteration, the method Section 6
 * compares CMCG against: time stepping with the source from u0_dev (NULL =
 * zero, as in the paper's experiments), one period after another, the state
 * at a period start being the iterate U_0^(l); its time-harmonic
 * approximation F_psi U_0^(l) (Section 5.4) comes from one final period with
 * the filter.  Options: o->fixed_iters = L > 0 simulates exactly L periods
 * (L - 1 plain ones, then the filtered one); otherwise the plain periods stop
 * once the state changes by at most o->tol between period starts,
 * ||U_0^(l) - U_0^(l-1)||_{eps,mu} / ||U_0^(l)||_{eps,mu}, or after
 * o->max_iter - 1 of them (CMCG_NOT_CONVERGED).  The result holds the
 * filtered field, U0 = the final iterate, the history of relative state
 * changes (one per plain period) and stats with iters = plain periods and
 * periods = plain periods + 1.  Uses the problem's work buffers: not
 * concurrently with another solve of the same problem. */
int cmcg_fw_solve(cmcg_problem* p, const cmcg_options* o, const double* u0_dev,
                  hipStream_t stream, cmcg_result** out);
/* Batched solve: Algorithm 3 for n problems sharing one space (same mesh,
 * order and field precision; each with its own omega, j, g and materials),
 * advanced together -- one kernel launch per Runge-Kutta stage covers every
 * member, members with shorter periods or a converged CG idle.  Each member
 * stops on its own tolerance; its result equals the one cmcg_solve returns
 * for it alone (same arithmetic and reduction order).  results[n] receives
 * one result per member (owned by the caller).  Returns CMCG_OK when every
 * member converged, CMCG_NOT_CONVERGED when some stopped at max_iter, or an
 * error (then no results; CMCG_ERR_ARG when the problems do not share a
 * space or a time scheme, or n > 65535: members are the launch's second grid
 * dimension). */
int cmcg_solve_batch(cmcg_problem* const* problems, int n, const cmcg_options* o,
                     hipStream_t stream, cmcg_result** results);
/* Filtered time-harmonic fields (complex amplitudes at the DG nodes),
 * [K][Np][3] each, host pointers; any output may be NULL. */
int cmcg_result_fields(const cmcg_result* r, double* e_re, double* e_im, double* h_re,
                       double* h_im);
/* Filtered field as device dof vectors [K][6][Np] FP64 (re, im); the first
 * harmonic of a several-frequency result. */
int cmcg_result_filtered_device(const cmcg_result* r, double* f_re_dev, double* f_im_dev,
                                hipStream_t stream);
/* Number of filtered harmonics in a result (1 for a single frequency), and
 * the filtered field of harmonic h (0 <= h < nh) as device dof vectors;
 * CMCG_ERR_ARG for h out of range. */
int cmcg_result_harmonics(const cmcg_result* r, int* nh);
int cmcg_result_filtered_harmonic_device(const cmcg_result* r, int h, double* f_re_dev,
                                         double* f_im_dev, hipStream_t stream);
/* The periodic initial condition U0 reached by CG, device dof vector. */
int cmcg_result_initial_device(const cmcg_result* r, double* u0_dev, hipStream_t stream);
int cmcg_result_stats(const cmcg_result* r, cmcg_stats* st);
/* ||R_l|| / ||R_0|| for l = 0..iters; copies min(cap, iters+1) values. */
int cmcg_result_history(const cmcg_result* r, double* rel_res, int cap, int* n);
void cmcg_result_destroy(cmcg_result* r);

/* ---------------------------------------------------------- debug hooks -- */
/* Per-kernel parity entry points.  Device dof vectors [K][6][Np] FP64 in and
 * out (converted to / from the space's precision inside), ordered on
 * `stream`, synchronous on return.
 *
 * cmcg_debug_rhs: out = Phi(t, U) = B U (+ Re(JJ e^{i omega t}) when
 *   with_source), the semi-discrete right-hand side of Section 5.2.2.
 * cmcg_debug_period: one period of M steps from U0 (Section 5.3): direction
 *   +1 = forward P (P_psi when with_source), -1 = adjoint P* = S P S (never
 *   with source).  f_re / f_im (may be NULL) receive the filtered field of
 *   a forward period (trapezoid for RK2, Hermite for RK4).
 * cmcg_debug_step: one time step (Section 5.3: RK2 for q = 1, classical RK4
 *   otherwise, or o->scheme) from t_m = m dt to t_{m+1}, dt = T / M with M
 *   the step count `o` selects (0 <= m < M, else CMCG_ERR_ARG): direction +1
 *   applies the forward step (with the source Re(JJ e^{i omega t}) at the
 *   stage times when with_source), -1 the adjoint step S R S (never with
 *   source).  This is exactly the launch sequence that a period repeats M
 *   times: FP32 spaces round the input to FP32 (+ bfloat16 low part) and
 *   return the compensated state.
 * cmcg_debug_dot: (U, V)_{eps,mu} = V^T M U (Section 2.2), into *out (host),
 *   with a fixed reduction order (bitwise reproducible). */
int cmcg_debug_rhs(cmcg_problem* p, const cmcg_options* o, double t, int with_source,
                   const double* u_dev, double* out_dev, hipStream_t stream);
int cmcg_debug_period(cmcg_problem* p, const cmcg_options* o, int direction,
                      int with_source, const double* u0_dev, double* ut_dev,
                      double* f_re_dev, double* f_im_dev, hipStream_t stream);
int cmcg_debug_step(cmcg_problem* p, const cmcg_options* o, int m, int direction, int with_source,
                    const double* u_dev, double* out_dev, hipStream_t stream);
int cmcg_debug_dot(cmcg_problem* p, const double* u_dev, const double* v_dev, double* out,
                   hipStream_t stream);
/* One 16x16x4 matrix-core product D = A B (v_mfma_f64_16x16x4f64 for
 * CMCG_FP64, v_mfma_f32_16x16x4f32 for CMCG_FP32 with the inputs rounded to
 * FP32) through the operand and accumulator lane layout the matrix-core stage
 * kernels assume.  a_dev [16][4], b_dev [4][16], d_dev [16][16]: row-major
 * FP64 device arrays; synchronous on return.  Errors: CMCG_ERR_ARG (NULL,
 * unknown precision). */
int cmcg_debug_mfma(int precision, const double* a_dev, const double* b_dev, double* d_dev, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the inner
 * product of cmcg_debug_dot, (U, V)_{eps,mu}, with the same kernels and
 * summation order (bit-for-bit the same value), written to *out_dev (device
 * memory, one double) in order on `stream`, without synchronising and
 * without allocating anything.  Its partial sums go to a fixed device array
 * of 1024 doubles (8 KB) that the library holds on every GPU it runs on until
 * the process ends; any K is accepted (the reduction uses at most 1024
 * partials; a size needing more would be rejected with CMCG_ERR_ARG).  Every
 * partial is written before it is read, so the array needs no clearing.
 * All calls on one GPU share that array: calls that may overlap on one GPU
 * (different streams without ordering between them, several host threads)
 * race and must be serialised by the caller.  u_dev, v_dev: device dof
 * vectors of p's space (FP64).  Errors: CMCG_ERR_ARG (NULL argument),
 * CMCG_ERR_STATE (p's device is not current), CMCG_ERR_DEVICE (launch). */
int cmcg_debug_dot_noalloc(const cmcg_problem* p, const double* u_dev, const double* v_dev,
                           double* out_dev, hipStream_t stream);

/* ------------------------------------------------------------ serving -- */
/* Continuous batching of independent solve requests (any mesh, order,
 * frequency, source).  Each admitted problem occupies a slot with its own
 * stream and runs exactly the launch sequence of cmcg_solve (Algorithms 1-3 +
 * filter period), so its result equals the one cmcg_solve returns.
 *
 * cmcg_problem_footprint: device bytes a solve of p keeps resident (problem
 *   data, field / filter / CG vectors, result) -- the admission cost; with
 *   local time stepping (o->lts_ratio > 1) the engine adds 12 field vectors
 *   and the fine-region masks and block lists.
 * cmcg_engine_create: budget = device bytes the engine may hold for admitted
 *   solves; max_slots = concurrent solves (1..1024).
 * cmcg_engine_admit: starts a solve in a free slot; CMCG_ERR_NOMEM when no
 *   slot is free, the footprint does not fit the remaining budget or a device
 *   allocation for the solve failed (the caller keeps the request queued; if
 *   the engine holds no other solve, waiting will not help),
 *   CMCG_ERR_TOO_LARGE when the footprint exceeds the whole budget (the
 *   request can never be admitted), CMCG_ERR_STATE when p is already held by
 *   a slot.  p must stay alive until the slot is collected or cancelled.
 * cmcg_engine_step: advances every running slot whose chunk of work (the
 *   initial periods, one half of a CG iteration, or the filter period) has
 *   completed on its stream, enqueueing its next chunk; waits (polling) until
 *   at least one slot has advanced, so slots of different sizes never wait
 *   for one another; reports how many slots still run and how many wait for
 *   collection.
 * cmcg_engine_poll: slot state 0 free, 1 running, 2 finished, 3 failed.
 * cmcg_engine_collect: hands over the result of a finished slot and frees it
 *   (returns the solve's status, or its error code for a failed slot).
 * cmcg_engine_cancel: stops a slot and frees it.
 * Not thread-safe; calls must come from one thread with the engine's device
 * current. */
typedef struct cmcg_engine cmcg_engine;
int cmcg_problem_footprint(const cmcg_problem* p, size_t* bytes);
int cmcg_engine_create(size_t hbm_budget, int max_slots, cmcg_engine** out);
void cmcg_engine_destroy(cmcg_engine* e);
int cmcg_engine_admit(cmcg_engine* e, cmcg_problem* p, const cmcg_options* o, int* slot);
int cmcg_engine_step(cmcg_engine* e, int* n_running, int* n_finished);
int cmcg_engine_poll(const cmcg_engine* e, int slot, int* state);
int cmcg_engine_collect(cmcg_engine* e, int slot, cmcg_result** out);
int cmcg_engine_cancel(cmcg_engine* e, int slot);
int cmcg_engine_info(const cmcg_engine* e, size_t* used, int* n_running, int* n_finished);
/* Co-batching: n (1..65535) requests on one space (same mesh, order and
 * field precision) admitted into one slot and solved together by the batched
 * path of cmcg_solve_batch (one launch per Runge-Kutta stage for every
 * member), so small requests fill the device together.  Each member's result
 * equals the one cmcg_solve returns for it alone.  The solve runs on a worker
 * thread that uses the slot's stream; the batch is set up and its periods
 * captured as graphs during this call, on the caller's thread (a capture
 * would refuse the caller's legacy-stream work from any other thread), and
 * the worker only replays them.  cmcg_engine_step reports the slot finished
 * once the solve has ended.  Admission cost: the members' summed
 * footprints plus what the batch copies: every member's source and source
 * mask (when any member has a source) and the geometry and mass weights
 * (once when the members share their media, else per member).  Errors as
 * cmcg_engine_admit, and CMCG_ERR_ARG when the
 * problems do not share a space, repeat, or ask for local time stepping.
 * o->progress is not called and o->autotune is ignored.
 * cmcg_engine_slot_members: members of a slot (0 free, 1 for a single solve).
 * cmcg_engine_collect_batch: hands over the n results of a finished
 *   co-batched slot (caller-owned) and frees the slot; returns
 *   CMCG_NOT_CONVERGED when a member stopped at max_iter, the batched solve's
 *   error code (no results) when it failed.  cmcg_engine_collect refuses a
 *   co-batched slot (CMCG_ERR_STATE); cmcg_engine_cancel stops its solve at
 *   the next CG iteration (after that iteration's periods and one filter
 *   period) and waits for the worker. */
int cmcg_engine_admit_batch(cmcg_engine* e, cmcg_problem* const* problems, int n, const cmcg_options* o,
                            int* slot);
int cmcg_engine_slot_members(const cmcg_engine* e, int slot, int* n);
int cmcg_engine_collect_batch(cmcg_engine* e, int slot, cmcg_result** results, int n);

/* ------------------------------------------------------------- tuning -- */
/* Stage-kernel implementation variant for (q, precision): 0 gathers each
 * face's neighbour traces when it is processed, 1 requests them one face
 * ahead (more registers, more latency hiding), 2 runs the volume and lift
 * products on the matrix cores (q = 2, 3; FP32 fields on
 * v_mfma_f32_16x16x4f32, FP64 fields on v_mfma_f64_16x16x4f64; q = 1 falls
 * back to 0), 3 is 2 with the neighbour traces requested one face ahead, 4
 * is 3 with two waves per 10-element block, each computing half of the
 * output tiles (q = 2, 3), 5 is 4 with the neighbour traces of all four
 * faces requested at once and two alternating flux tiles (q = 2, 3), 6 is 4
 * with the two waves splitting the output by column tiles instead of row
 * tiles (q = 3), 7 combines 5 and 6 (q = 3), 8 is 3 with four waves per
 * block, each computing one row tile and half of the column tiles (q = 3)
 * or a quarter of them (q = 2), 9 is 8 with the neighbour traces of all four
 * faces requested at once (q = 2, 3; more registers per wave: for launches
 * of a round of workgroups or less); variants that do not exist for
 * (q, precision) fall back to 0; -1 chooses per launch from its size
 * (workgroups of 10 elements over all members), the form the autotuner's
 * timings favour there.  All compute the same Phi(t, Y) and stage update.
 * Local time stepping's substep launches (restricted to the element blocks
 * near the fine region) take the four-wave form whatever the choice.
 * Defaults: -1 for q = 2, 3, 0 for q = 1.  Process-wide;
 * not thread-safe against concurrent solves.  Returns CMCG_ERR_ARG for an unknown q / precision /
 * variant.  cmcg_tune_get_stage reports the current choice (possibly -1);
 * cmcg_tune_resolve_stage the variant a launch over K elements and
 * `members` members would run under it. */
#define CMCG_STAGE_VARIANTS 10
int cmcg_tune_stage(int q, int precision, int variant);
int cmcg_tune_get_stage(int q, int precision, int* variant);
int cmcg_tune_resolve_stage(int q, int precision, int64_t K, int members, int* variant);

/* Autotuner: times every stage-kernel variant that applies to p's (q,
 * precision) on p's own launch shape -- up to 8 homogeneous time steps on
 * its mesh and work buffers (o's scheme and step rule; o may be NULL), one
 * warm-up run and the best of two timed runs (HIP events on `stream`) per
 * variant -- keeps the fastest as the process-wide choice for (q, precision)
 * (as cmcg_tune_stage does) and returns it in *variant.  us_per_launch
 * (nullable, CMCG_STAGE_VARIANTS entries) receives each variant's average
 * stage-launch time in microseconds, 0 for variants that do not apply.  Overwrites p's work
 * buffers, not its data; must not overlap a solve of p or any solve of the
 * same (q, precision).  Errors: CMCG_ERR_ARG (NULL p or variant), device
 * errors as CMCG_ERR_DEVICE. */
int cmcg_autotune_stage(cmcg_problem* p, const cmcg_options* o, hipStream_t stream, int* variant,
                        double* us_per_launch);
/* The same for a batch (the shape cmcg_solve_batch launches): the n problems
 * must satisfy cmcg_solve_batch's rules; every variant that applies is timed
 * on up to 8 homogeneous time steps of the batched launch with every member
 * active (one launch per Runge-Kutta stage covers all members), the fastest
 * is kept as the process-wide choice for (q, precision) and remembered for
 * (device, q, precision, K, n), so a later cmcg_solve_batch with
 * o->autotune = 1 reuses it.  us_per_launch (nullable, CMCG_STAGE_VARIANTS
 * entries): average microseconds per batched stage launch, 0 where a variant
 * does not apply.  Allocates the batch's working set for the duration of the
 * call; does not change the problems' data.  Errors as cmcg_solve_batch;
 * CMCG_ERR_ARG for 2-D spaces (one 2-D stage kernel). */
int cmcg_autotune_batch(cmcg_problem* const* problems, int n, const cmcg_options* o, hipStream_t stream,
                        int* variant, double* us_per_launch);

#ifdef __cplusplus
}
#endif
#endif /* CMCG_H */
