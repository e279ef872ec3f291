/*
 * hlbm.h -- C ABI of the MI355X (gfx950) library for the moving-grid hybrid
 * lattice Boltzmann method (MG-HLBM) of Di Ilio, Chiappini, Ubertini, Bella
 * and Succi, "A moving-grid approach for fluid-structure interaction problems
 * with hybrid lattice Boltzmann method" (arXiv 2006.13631).
 *
 * The library advances a thin rigid lamina oscillating as y(t) = A sin(omega t)
 * in a fluid at rest (Sec. Problem statement): a D2Q9 BGK background lattice
 * (Eq.(LBE), Eq.(local_eq)), a body-fitted triangular grid that moves with the
 * lamina and is advanced with the cell-vertex finite-volume scheme Eq.(ulbe)
 * in n sub-steps per lattice step, the two-way exchange of Eqs.
 * (postcollision2_s) and (postcollision2_u), the refill of the moved grid
 * (Sec. Refill procedure), and the force on the lamina from which the
 * hydrodynamic function Theta of Eq.(force_phasor) is fitted (Sec. 2.1).
 *
 * Conventions for every call:
 *  - Return 0 on success or a negative HLBM_E_* code; no exception or signal
 *    crosses the ABI. Output arguments are written only on success.
 *  - Host pointers belong to the caller and are only read or written during
 *    the call. Device memory belongs to the library (allocated in
 *    hlbm_create, released in hlbm_destroy).
 *  - A handle is used by one host thread at a time. Results are
 *    deterministic: the same configuration and call sequence give the same
 *    bits on the same GPU.
 *  - Lattice units: lattice spacing and structured time step are 1, reference
 *    density 1, c_s^2 = 1/3.
 */
#ifndef HLBM_H
#define HLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------ */
#define HLBM_OK 0
#define HLBM_E_ARG -1         /* invalid argument or configuration          */
#define HLBM_E_NOMEM -2       /* device or host allocation failed           */
#define HLBM_E_HIP -3         /* HIP runtime error (text in hlbm_last_error) */
#define HLBM_E_UNSTABLE -4    /* a non-finite force or density was detected  */
#define HLBM_E_STATE -5       /* call not valid in the handle's state        */
#define HLBM_E_UNSUPPORTED -6 /* option not implemented in this build        */

/* ---- background lattice boundaries ------------------------------------ */
#define HLBM_BC_PERIODIC_X_WALLS_Y 0 /* periodic in x; halfway bounce-back walls
                                        at rest at y = -1/2 and y = ny - 1/2 */
#define HLBM_BC_PERIODIC 1           /* periodic in x and y                  */
#define HLBM_BC_PAPER 2              /* the paper's outer boundaries (Sec.
                                        Problem statement): no-slip walls at
                                        x = -1/2, nx - 1/2 (halfway bounce-
                                        back) and zero-gradient outflow at the
                                        y ends                                */
#define HLBM_BC_RING 3               /* finest level of a multi-level handle
                                        only: the outermost ring of nodes is
                                        written from the next coarser level   */

/* ---- storage of the lattice populations ------------------------------- */
#define HLBM_FP64 0     /* FP64 storage and arithmetic                          */
#define HLBM_FP32 1     /* FP32 storage and arithmetic                          */
#define HLBM_FP16_DEV 2 /* FP16 storage of f_i - w_i, FP32 arithmetic           */

/* ---- flags ------------------------------------------------------------- */
#define HLBM_FLAG_NO_BODY 1 /* grid without the lamina slot; b still sets A and
                               omega (used to check the moving-grid coupling) */

/* ---- state selectors for hlbm_get_state / hlbm_set_state --------------- */
#define HLBM_STATE_LATTICE 0 /* double [9][ny][nx]: post-collision f at t_k     */
#define HLBM_STATE_GRID 1    /* double [9][nux*nuy]: grid f at t_k, node
                                index j*nux + i                              */
#define HLBM_STATE_ADJ_LATTICE 2 /* get only, double [9][ny][nx]: dJ/d(lattice
                                    at t_0) from the last hlbm_adjoint       */
#define HLBM_STATE_ADJ_GRID 3    /* get only, double [9][nux*nuy]: dJ/d(grid at
                                    t_0) from the last hlbm_adjoint          */
#define HLBM_STATE_MOTION 4      /* get only, double [steps][2]: (y, v) of a
                                    coupled lamina after each step, entry k
                                    at t = k+1 (hlbm_set_motion)              */
#define HLBM_STATE_LEVEL 16      /* + l: double [9][ny_l][nx_l], post-collision f
                                    of refinement level l of a multi-level
                                    handle (l = nlevels-1 is the finest, also
                                    HLBM_STATE_LATTICE)                       */

/* Problem and discretisation (Sec. Problem statement, Sec. HLBM).
 * Grid node (i, j) sits at x = nx/2 + (i - nux/2) h_u (integer division) and
 * y = (ny-1)/2 + y(t) + (j - (nuy-1)/2) h_u; the lamina of width b and
 * thickness h_u fills the slot between rows nuy/2-1 and nuy/2 for
 * |x - nx/2| <= b/2. Derived quantities:
 *   nu = (tau - 1/2)/3, tau_u = tau - 1/2, A = kc b / (2 pi),
 *   omega = 2 pi nu beta / b^2, n = n_sub, or when n_sub = 0
 *   n = max(2, ceil(1/tau_u - 1e-9)), Delta t_u = 1/n. */
typedef struct hlbm_config {
  int32_t nx, ny;     /* background lattice nodes                         */
  int32_t nux, nuy;   /* body-fitted grid nodes; nuy even                 */
  double h_u;         /* grid spacing in lattice units (0: 1)             */
  double b;           /* lamina width L                                   */
  double thickness;   /* lamina thickness T; must equal h_u               */
  double tau;         /* structured relaxation time tau_s (> 1/2)         */
  double kc;          /* Keulegan-Carpenter number 2 pi A / L             */
  double beta;        /* frequency parameter omega L^2 / (2 pi nu)        */
  int32_t n_sub;      /* grid sub-steps per lattice step (0: automatic)   */
  int32_t bc;         /* HLBM_BC_*                                        */
  int32_t storage;    /* HLBM_FP64 | HLBM_FP32 | HLBM_FP16_DEV            */
  int32_t flags;      /* HLBM_FLAG_*                                      */
  int32_t ckpt_every; /* adjoint checkpoint window (0: no adjoint)        */
  int32_t reserved;   /* must be 0                                        */
  int64_t max_steps;  /* capacity of the force history (steps)           */
} hlbm_config;

/* Derived parameters and counters of a case. */
typedef struct hlbm_info {
  double nu, tau_u, dt_u, A, omega, period, u_max, mach, reynolds, eps;
  int32_t n_sub, nnode, ntri, n_interface, n_wall, n_wall_edges;
  int32_t beta_limit_ok; /* 1 if beta < 2.6 eps^-1.6, Eq.(betalimit) */
  int32_t n_classes;     /* distinct finite-volume stencils on the grid */
  int64_t step;          /* structured steps taken                      */
  double y;              /* lamina offset y(t_k)                         */
  int64_t n_type1, n_type2, n_type3; /* refill counts, summed over steps */
  int64_t lattice_bytes; /* device bytes of one lattice buffer          */
  int32_t status;        /* HLBM_STATUS_*                               */
  int32_t two_step;      /* 1: pairs of steps advance the lattice away
                            from the grid in one launch (the band near it
                            one step at a time); same results either way */
} hlbm_info;

#define HLBM_STATUS_RUNNING 0  /* steps left                                  */
#define HLBM_STATUS_DONE 1     /* max_steps reached                            */
#define HLBM_STATUS_UNSTABLE 2 /* a non-finite force appeared; the case stopped */

/* Schedule of a handle, chosen by hlbm_tune. None of the choices changes
 * any result: every case computes the same bits. A single case uses the
 * stream-collide shape and order and the sub-step variant. */
typedef struct hlbm_tuning {
  int32_t steps_per_graph; /* structured steps captured in one HIP graph
                              (batch)                                      */
  int32_t lattice_threads; /* stream-collide workgroup width: 64..256, a
                              multiple of 64                               */
  int32_t lattice_rows;    /* lattice rows per lane of the stream-collide:
                              1, 2 or 4                                    */
  int32_t substep_variant; /* grid sub-step kernel (grid nodes per tile,
                              workgroup size): -1 default (FP64 1, else
                              3); 0: 16x16, 576; 1: 32x8, 640; 2: 64x4,
                              896; 3: 16x8, 384; 4: 8x8, 64; 5: 16x8,
                              128; 6: 16x16, 256; 7: 8x4, 64 (4-7: several
                              nodes per lane, more workgroups per CU),
                              each up to 4 sub-steps per launch; single
                              case only: 8: 32x8, 256 and 9: 16x16, 256,
                              one sub-step per launch; 10: 32x8, 384, two
                              (large grids)                                */
  int32_t order;           /* batch work lists: 0 case by case, 1 dealt to
                              the 8 XCDs in contiguous chunks; single
                              case: bit 0 gives each XCD a contiguous band
                              of stream-collide rows, bit 1 deals the
                              two-step tiles to the XCDs in contiguous
                              runs, each XCD starting at its own offset    */
  int32_t tail_variant;    /* batch: sub-step variant once at most
                              max(1, ncases/8) cases still run (-1: the
                              same as substep_variant); single case: -1    */
  int32_t persistent;      /* batch: 0 HIP graphs of steps_per_graph steps;
                              1 one cooperative launch per run of up to
                              256 steps, every workgroup walking the
                              kernels of a step with a grid-wide barrier
                              between them; 2 graphs, then the cooperative
                              launch once at most max(1, ncases/8) cases
                              run. The cooperative launch takes sub-step
                              variants 4-7 (others: 5) and one lattice row
                              per lane; single case: 0                     */
  int32_t persistent_groups; /* batch: workgroups of the cooperative launch
                              (0: as many as the widest kernel of a step
                              has work items, at most what fits at once)   */
  double ms_per_step;      /* measured for the chosen schedule (output)      */
} hlbm_tuning;

typedef struct hlbm hlbm_t;

/* Create a case: validate the configuration, build the grid and its
 * finite-volume matrices S_ik, C_ik (median-dual control volumes, Eq.(ulbe)),
 * allocate device buffers and set both grids to rest (f = w_i).
 * ncases > 1 creates a batch: cfg points to ncases configurations (sizes,
 * KC, beta, tau, n_sub may all differ; storage must be the same, ckpt_every
 * 0, every case with a grid), advanced together by case-batched kernels.
 * In a batch, case_id selects the case in hlbm_force, hlbm_info_get and
 * hlbm_get/set_state; hlbm_step advances every running case and lets each
 * stop at its own max_steps (or when its force becomes non-finite, status
 * HLBM_STATUS_UNSTABLE) instead of failing. Errors: HLBM_E_ARG (invalid
 * configuration: tau <= 1/2, Delta t_u >= 2 tau_u, grid or its motion
 * leaving the lattice, lamina not inside the fictitious rectangle,
 * |A omega| >= 1; in a batch, mixed storage or ckpt_every != 0),
 * HLBM_E_NOMEM, HLBM_E_HIP. On error *out is set to NULL. */
int hlbm_create(const hlbm_config *cfg, int32_t ncases, hlbm_t **out);

/* ---- structured refinement levels ------------------------------------ */
/* The paper divides the structured domain into refinement levels (Sec.
 * Problem statement: four levels, the relaxation time given on the finest)
 * and prints no interface scheme; the one built here: level l+1 covers the
 * node box box[l] = (x0, y0, x1, y1) of level l (inclusive) with twice the
 * resolution, 2 (x1-x0) + 1 by 2 (y1-y0) + 1 nodes, coinciding with level l
 * at every other node. Each level steps with Delta t = Delta x (acoustic
 * scaling), two steps per step of the next coarser level, and relaxes with
 * tau_l - 1/2 = (tau_fine - 1/2) / 2^(L-1-l) (equal viscosity). At the
 * interfaces the pre-collision density, velocity and f^neq = f - f^eq are
 * exchanged, f^neq scaled by the ratio of tau Delta x of the two levels
 * (first-order Chapman-Enskog), and written as post-collision populations
 * f^eq + (1 - 1/tau) f^neq: the ring of level l+1 before each of its steps,
 * linear along the box perimeter between level-l nodes and linear in time
 * between level l's states at t and t+1; level l's nodes one inside the box
 * after every second step of level l+1. */
#define HLBM_MAX_LEVELS 8
typedef struct hlbm_levels {
  int32_t nlevels;  /* 2 .. HLBM_MAX_LEVELS                                */
  int32_t nx0, ny0; /* level-0 lattice nodes                               */
  int32_t bc0;      /* boundaries of level 0: HLBM_BC_PERIODIC_X_WALLS_Y,
                       HLBM_BC_PERIODIC or HLBM_BC_PAPER                   */
  int32_t box[HLBM_MAX_LEVELS - 1][4]; /* box[l]: x0, y0, x1, y1 in level-l
                       nodes; 2 <= x0, x0 + 4 <= x1 <= nx_l - 3, same in y */
} hlbm_levels;

/* Create a multi-level handle. `fine` configures the finest level in its own
 * lattice units (tau, the lamina and its grid, storage, max_steps counted in
 * finest steps): nx and ny must be the shape the last box implies, bc must
 * be HLBM_BC_RING and ckpt_every 0; the grid and its motion must stay
 * inside the finest level (the geometric checks of hlbm_create). Every
 * level starts at rest. On the handle, hlbm_step(h, n) advances level 0 by
 * n steps (level l by n 2^l); hlbm_force, hlbm_info_get and
 * hlbm_get_stencil report the finest level's case; hlbm_get/set_state take
 * HLBM_STATE_LEVEL + l (set: the level's state is taken as steady, both of
 * its time levels get it), HLBM_STATE_LATTICE and HLBM_STATE_GRID for the
 * finest level; hlbm_tune tunes the finest level's kernels and applies its
 * stream-collide shape to every level. hlbm_adjoint and hlbm_timing return
 * HLBM_E_UNSUPPORTED. Errors: HLBM_E_ARG (invalid levels or boxes, or a
 * finest configuration hlbm_create would reject), HLBM_E_NOMEM, HLBM_E_HIP. */
int hlbm_create_multilevel(const hlbm_config *fine, const hlbm_levels *levels,
                           hlbm_t **out);

/* Shape and relaxation time of level `level` of a multi-level handle.
 * HLBM_E_STATE on another handle, HLBM_E_ARG for a level out of range. */
int hlbm_level_shape(hlbm_t *h, int32_t level, int32_t *nx, int32_t *ny,
                     double *tau);

/* ---- graded body-fitted grid ------------------------------------------ */
/* A single case whose grid has graded spacing (the paper refines its
 * unstructured grid toward the body): column i of the grid at local
 * x = x_nodes[i], row j at local y = y_nodes[j] (lamina centre at the
 * origin; both strictly increasing, the rows symmetric about the lamina,
 * y_nodes[j] = -y_nodes[nuy-1-j]); each cell is cut along the diagonal of
 * its side of the centre as in the uniform grid, the lamina fills the cells
 * of row nuy/2-1 inside |x| <= b/2, and cfg->thickness must equal
 * y_nodes[nuy/2] - y_nodes[nuy/2-1]. h_u is not used for the grid. The
 * finite-volume matrices follow the cells' own sizes; the fictitious
 * rectangle is the grid's bounding box inset by 2. Otherwise as
 * hlbm_create with ncases = 1 (the geometric checks use the grid's
 * extents), checkpoints and hlbm_adjoint included: the derivatives of the
 * interpolation weights in y_k follow each cell's own height. */
int hlbm_create_graded(const hlbm_config *cfg, const double *x_nodes,
                       const double *y_nodes, hlbm_t **out);

/* A single case on any triangulation of the grid region (Sec. Hybrid
 * lattice Boltzmann method: the body-fitted grid is an unstructured
 * triangular mesh around the body). Nodes at local coordinates
 * xy[2 p], xy[2 p + 1] (lamina centre at the origin), node_type[p] one of
 * 0 (discretization), 1 (interface: the grid's outer boundary), 2 (wall:
 * the lamina's surface), triangles tri[3 t .. 3 t + 2] counter-clockwise;
 * host arrays, read during the call only. The grid must cover its
 * bounding box (symmetric about y = 0) minus the lamina |x| < b/2,
 * |y| < cfg->thickness/2: every edge of one triangle joins two interface
 * nodes or two wall nodes, interface nodes lie on the bounding box. Each
 * node's stencil holds the vertices of the triangles around it, with the
 * median-dual matrices of Eq.(ulbe) (Sec. Hybrid lattice Boltzmann
 * method); points are located in unit buckets, the lowest-numbered
 * triangle holding a point within 1e-12 in each barycentric coordinate
 * taking it; the sub-steps run one per launch; a lattice node the grid
 * does not cover stops the case (flag bit 4, HLBM_E_UNSTABLE). The
 * fictitious rectangle is the bounding box inset by 2; nux, nuy and h_u
 * are not used. Otherwise as hlbm_create with ncases = 1. ckpt_every must
 * be 0 (no adjoint). Errors: HLBM_E_ARG (invalid mesh or configuration,
 * hlbm_last_error(NULL) says which), HLBM_E_NOMEM, HLBM_E_HIP. */
int hlbm_create_mesh(const hlbm_config *cfg, int32_t nnode, const double *xy,
                     const int32_t *node_type, int32_t ntri, const int32_t *tri,
                     hlbm_t **out);

/* A bending lamina on a given triangulation (the extension to deformable
 * bodies that Sec. Conclusions names; the paper's lamina is rigid). The
 * centreline moves as A sin(omega t) + B sin(omega t + phi) (2x/b)^2 for
 * |x| <= b/2, and the grid follows: node p, at local (x_p, y_p) in the
 * triangulation given to hlbm_create_mesh, sits at y_p + s(x_p) w(y_p)
 * beta_k during step k, beta_k = B sin(omega k + phi), where s is
 * (2x/b)^2 on the lamina and falls linearly to 0 at the grid's left and
 * right sides, and w is 1 for |y| <= thickness/2 and falls linearly to 0
 * at its top and bottom, so the outer boundary moves rigidly and the
 * lamina keeps its thickness. Every step first rebuilds the grid's
 * finite-volume matrices, triangles and wall edges for the configuration
 * beta_k (one launch); the sub-steps impose the wall velocity
 * A omega cos(omega t) + B omega cos(omega t + phi) s(x); the refill
 * locates a node's position of t_{k+1} in the grid of t_k and keeps f
 * (type 2) inside the bent lamina |y - beta_k (2x/b)^2| < thickness/2;
 * the force integrates over the bent wall edges. hlbm_stencil returns the
 * weights of the last configuration (that of t_0 before the first step).
 * Call before the first step of a single case from hlbm_create_mesh with
 * the lamina. Needs |B| < 1, the bent lamina (thickness/2 + |B| + 1) at
 * least one lattice unit inside the fictitious rectangle, |A omega| +
 * |B omega| < 1, and every triangle keeping a positive area at beta =
 * +-B. Errors: HLBM_E_UNSUPPORTED (not such a case), HLBM_E_STATE (steps
 * taken, coupled motion, no lamina), HLBM_E_ARG (B or phi out of range,
 * hlbm_last_error says which), HLBM_E_HIP. A bending case takes no
 * coupled motion. */
int hlbm_set_deformation(hlbm_t *h, double B, double phi);

/* ---- two-way coupled motion ------------------------------------------- */
/* The paper prescribes the lamina's motion (Sec. Problem statement: known a
 * priori). Instead, the lamina may be mounted on a spring and damper and
 * moved by the fluid: M y'' + C y' + K y = F_y per unit depth, F_y the
 * wall force of each step. Advanced once per step by semi-implicit Euler
 * with Delta t = 1 (v_{k+1} = v_k + (F_y(t_{k+1}) - K y_k - C v_k)/M, then
 * y_{k+1} = y_k + v_{k+1}); during the sub-steps of step k the wall moves
 * with v_k. On the device: the force kernel updates the state and writes
 * the next step's offset, fictitious rectangle and wall velocities. */
typedef struct hlbm_motion {
  double mass;      /* M > 0, per unit depth (lattice units, rho0 = 1)    */
  double stiffness; /* K >= 0                                            */
  double damping;   /* C >= 0                                            */
  double y0, v0;    /* state at t_0: |y0| <= y_max, |v0| < 1             */
  double y_max;     /* bound on |y|: the grid and its lattice donors must
                       stay inside the lattice for every |y| <= y_max (the
                       checks of hlbm_create with y_max for |A|); a state
                       beyond it, or |v| >= 1, stops the case:
                       HLBM_E_UNSTABLE                                    */
} hlbm_motion;

/* Switch a single case with a lamina to coupled motion, before its first
 * step (kc and beta then play no part). hlbm_force keeps fitting Theta
 * only where the caller's omega applies; the motion is read with
 * hlbm_get_state(HLBM_STATE_MOTION). Errors: HLBM_E_STATE (steps already
 * taken, no lamina), HLBM_E_ARG (invalid parameters or bound),
 * HLBM_E_UNSUPPORTED (a batch or multi-level handle). hlbm_adjoint of a
 * coupled case returns HLBM_E_UNSUPPORTED. */
int hlbm_set_motion(hlbm_t *h, int32_t case_id, const hlbm_motion *m);

/* Advance nsteps structured steps t_k -> t_{k+1} (Sec. HLBM and Sec. Refill
 * procedure): lattice interpolation nodes from the grid (Eq.
 * (postcollision2_s)), lattice stream-collide (Eq.(LBE)), n grid sub-steps
 * (Eq.(ulbe), Eq.(postcollision2_u)), force, move and refill. Blocks until
 * the steps are done. HLBM_E_ARG if the force history would overflow
 * max_steps; HLBM_E_UNSTABLE if a non-finite force appeared. */
int hlbm_step(hlbm_t *h, int64_t nsteps);

/* The steps of hlbm_step (Sec. HLBM and Sec. Refill procedure), enqueued on
 * the handle's stream without waiting for them: the call returns once they
 * are launched. The status it returns covers the steps known to have
 * finished (the device flag as copied after an earlier hlbm_step_async, if
 * that copy is done): HLBM_E_UNSTABLE as hlbm_step reports it; a flag raised
 * by steps still running is reported by a later hlbm_step_async, hlbm_sync or
 * hlbm_step. Every other call on the handle first waits for the enqueued
 * steps. HLBM_E_ARG as hlbm_step (nothing is enqueued then). Single cases;
 * a batched or multi-level handle, and a single case with timing on, step
 * as hlbm_step does (blocking). */
int hlbm_step_async(hlbm_t *h, int64_t nsteps);

/* Wait for every step enqueued on the handle; returns what hlbm_step would
 * have returned for them (0, or HLBM_E_UNSTABLE with the cause in
 * hlbm_last_error). */
int hlbm_sync(hlbm_t *h);

/* Force history and hydrodynamic function (Sec. 2.1, Eq.(force_phasor)).
 * hist_xy (may be NULL) receives up to cap (Fx, Fy) pairs, entry k at
 * t = k+1; *n_out (may be NULL) gets the number of entries. If theta is not
 * NULL, F_y is fitted as a_s sin(omega t) + a_c cos(omega t) over
 * win_t0 <= t/T < win_t1 (T = 2 pi/omega; the paper uses [1, 4)) and
 * theta = (a_s, a_c) / ((pi/4) omega^2 b^2 A). HLBM_E_ARG if the window
 * holds fewer than two samples. */
int hlbm_force(hlbm_t *h, int32_t case_id, double *hist_xy, int64_t cap,
               int64_t *n_out, double win_t0, double win_t1, double theta[2]);

/* Discrete adjoint of the whole run (reverse mode over the steps taken so
 * far, every step of the method differentiated as the forward computed it).
 * For J = sum_k (dJ_dF[2k] F_x(t_{k+1}) + dJ_dF[2k+1] F_y(t_{k+1})), n = the
 * number of steps taken since creation, grad_A_omega_tau receives dJ/dA,
 * dJ/domega and dJ/dtau with A, omega and tau = tau_s independent (tau_u =
 * tau_s - 1/2 follows tau_s; kc and beta are only the way the configuration
 * names A and omega). The discrete decisions of the run (node status, donor
 * cells, triangles, refill types, n) are held fixed, so the result is the
 * derivative of the piecewise-smooth J on the run's piece.
 * Uses the checkpoints taken every ckpt_every steps during hlbm_step and
 * recomputes each window of steps into a device tape of
 * (ckpt_every + 1) lattice and ckpt_every (n + 1) + 1 grid arrays before
 * running it backwards; the adjoint of the initial state is kept for
 * hlbm_get_state (HLBM_STATE_ADJ_*). Blocks until done; the forward state
 * is left as it was. Errors: HLBM_E_STATE (no grid, ckpt_every = 0, or the
 * state was replaced by hlbm_set_state after step 0), HLBM_E_ARG (n is not
 * the number of steps taken, or NULL pointers), HLBM_E_UNSUPPORTED (the
 * lattice donors of the grid wrap across a periodic y boundary),
 * HLBM_E_NOMEM (the tape does not fit: use a smaller ckpt_every). */
int hlbm_adjoint(hlbm_t *h, int32_t case_id, const double *dJ_dF, int64_t n,
                 double grad_A_omega_tau[3]);

/* Copy a state array to or from host memory, converted to or from FP64.
 * which = HLBM_STATE_* (the adjoint states can only be read, after
 * hlbm_adjoint; HLBM_E_STATE before); bytes must equal the array size in
 * doubles times 8 (HLBM_E_ARG otherwise). Setting a state after step 0
 * invalidates the checkpoints of a case created with ckpt_every > 0. */
int hlbm_get_state(hlbm_t *h, int32_t case_id, int32_t which, void *host_buf,
                   size_t bytes);
int hlbm_set_state(hlbm_t *h, int32_t case_id, int32_t which,
                   const void *host_buf, size_t bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * as hlbm_get_state for which = HLBM_STATE_LATTICE or HLBM_STATE_GRID (the
 * same bits), but it calls no hipMalloc, hipFree or other allocating
 * routine. hlbm_get_state converts the state to FP64 in a device buffer it
 * allocates for the call; this variant converts one population plane at a
 * time, in pieces of at most HLBM_NOALLOC_SCRATCH_BYTES, in a static device
 * buffer of that size which each GPU the library runs on holds until the
 * process ends, and copies each piece to host_buf before converting the
 * next, so a state of any size is read and no size exceeds the buffer.
 * Every call on a GPU shares that GPU's buffer: calls that overlap on one
 * GPU (from several host threads) race and must be serialized by the
 * caller. Blocks until the copy is done. Errors: HLBM_E_ARG (another
 * selector, a case_id out of range, NULL host_buf, or bytes not 8 times the
 * array's size in doubles), HLBM_E_STATE (HLBM_STATE_GRID of a case without
 * a grid), HLBM_E_HIP (the device address of the buffer could not be
 * obtained, or a copy failed). A multi-level handle reads its finest level
 * and grid; its coarser levels are not read this way. */
#define HLBM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20) /* 64 MiB per GPU */
int hlbm_get_state_noalloc(hlbm_t *h, int32_t case_id, int32_t which,
                           void *host_buf, size_t bytes);

/* Derived parameters and counters. */
int hlbm_info_get(hlbm_t *h, int32_t case_id, hlbm_info *out);

/* The grid's finite-volume matrices as assembled for the GPU, dense per node:
 * nbr [nnode][kmax] (-1 padded, slot 0 = the node itself), S [nnode][9][kmax]
 * streaming matrix S_ik, C [nnode][kmax] collision matrix C_ik (Eq.(ulbe)).
 * HLBM_E_ARG if kmax is smaller than the largest stencil. */
int hlbm_get_stencil(hlbm_t *h, int32_t kmax, int32_t *nbr, double *S,
                     double *C);

/* Per-kernel timing with HIP events recorded on the stream each kernel is
 * launched on. hlbm_timing(h, level) clears the accumulators and, for later
 * hlbm_step and hlbm_adjoint calls, records: level 1, every kernel of the
 * step (events between all kernels); level 2, the stream-collide alone, by
 * events taken at that kernel's own start and end and nothing else in the
 * step; level 3 (a case with a grid), each grid sub-step launch of
 * every step (of one step of every pair on the two-step path; at most 16
 * per step) the same way;
 * 0 turns recording off. Timed steps are launched one by one instead of as
 * graphs. hlbm_timing_get returns for kernel id (HLBM_K_*) the summed
 * milliseconds and launch count. HLBM_E_STATE for level 3 without a grid. */
#define HLBM_K_STREAM_COLLIDE 0 /* lattice stream-collide, Eq.(LBE)            */
#define HLBM_K_LATTICE_FROM_GRID 1 /* Eq.(postcollision2_s)                    */
#define HLBM_K_GRID_SUBSTEPS 2  /* donors + n sub-steps, Eqs.(ulbe),(postcollision2_u) */
#define HLBM_K_REFILL 3         /* move + refill                               */
#define HLBM_K_FORCE 4          /* wall force                                  */
#define HLBM_K_STEP 5           /* whole structured step                       */
#define HLBM_K_ADJ_STREAM_COLLIDE 6 /* adjoint of the lattice stream-collide   */
#define HLBM_K_ADJOINT 7        /* whole hlbm_adjoint call (count = steps)     */
#define HLBM_K_SUBSTEP_LAUNCH 8 /* level 3: each grid sub-step launch of a step
                                   (up to 16 per step; up to 4 sub-steps each,
                                   Eq.(ulbe)), count = launches timed        */
#define HLBM_K_ADJ_SUBSTEPS 9   /* hlbm_adjoint with timing on: the first
                                   reverse grid sub-step launch of every step
                                   (up to 4 sub-steps backwards), by events at
                                   its own start and end; count = launches  */
int hlbm_timing(hlbm_t *h, int32_t on);
int hlbm_timing_get(hlbm_t *h, int32_t kernel, double *total_ms, int64_t *count);

/* Autotuner. Batched handle: before its first step, time candidate
 * schedules for trial_steps steps of the whole batch, one choice at a time
 * (steps per graph 4/8/16; stream-collide shape 128/256 x 1/2/4 rows;
 * sub-step variant; work-list order; the cooperative launch in variants
 * 4-7, then its workgroup count) with the others held at the best so
 * far, then the sub-step variant and the launch kind on the
 * longest-running max(1, ncases/8) cases alone (tail_variant, persistent
 * 2), keep the fastest and restore the initial state. Single case (any
 * time, state untouched): time trial_steps launches of the stream-collide
 * in each shape and order, of the two-step stream-collide in each tile
 * order (where the case takes two steps per launch) and of one step's
 * sub-steps in each variant, reading the current lattice and grid and
 * writing only their free buffers, and keep the fastest (ms_per_step: the two chosen kernels' time per step).
 * trial_steps = 0 applies *t as given instead (single case: lattice_threads
 * = lattice_rows = 0 keeps the stream-collide shape). A single case then
 * captures the HIP graphs its next steps replay, so later hlbm_step calls
 * only launch them. *t receives the
 * schedule in use. Errors: HLBM_E_STATE (batch: steps already taken),
 * HLBM_E_ARG (invalid schedule). */
int hlbm_tune(hlbm_t *h, int32_t trial_steps, hlbm_tuning *t);

/* Release the device memory and streams of the handle (NULL is a no-op). */
void hlbm_destroy(hlbm_t *h);

/* Text of the last error on this handle, or of the last failed
 * hlbm_create when h is NULL. Valid until the next call on the handle. */
const char *hlbm_last_error(const hlbm_t *h);

#ifdef __cplusplus
}
#endif
#endif
