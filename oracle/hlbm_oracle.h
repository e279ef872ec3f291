/*
 * hlbm_oracle.h -- plain FP64 CPU oracle of the moving-grid hybrid lattice
 * Boltzmann method (MG-HLBM) of Di Ilio, Chiappini, Ubertini, Bella and Succi,
 * "A moving-grid approach for fluid-structure interaction problems with hybrid
 * lattice Boltzmann method" (arXiv 2006.13631).
 *
 * TEST INFRASTRUCTURE. This library exists only to check the GPU library.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it. It shares no code, header, table or helper with the
 * GPU path and is never a fallback for it.
 *
 * Everything is FP64, single-threaded, written as plain loops in the order the
 * paper states the method. Where the paper leaves a point open, the reading
 * taken is stated next to the code that takes it.
 */
#ifndef HLBM_ORACLE_H
#define HLBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* boundary conditions of the background lattice */
#define OR_BC_PERIODIC_X_WALLS_Y 0 /* periodic in x, halfway bounce-back walls at y=-1/2, ny-1/2 */
#define OR_BC_PERIODIC 1           /* periodic in x and y */
#define OR_BC_PAPER 2              /* the paper's outer boundaries (Sec. Problem statement):
                                      no-slip walls at x=-1/2, nx-1/2 (halfway bounce-back),
                                      zero-gradient outflow at the y ends */
#define OR_BC_RING 3               /* the outermost ring of nodes is given from outside
                                      (a refinement level fed by the next coarser one):
                                      ring nodes are not updated, every other node pulls
                                      from inside the lattice */

/* mesh node roles (Sec. Refill procedure) */
#define OR_NODE_INTERIOR 0  /* discretization node of the body-fitted grid      */
#define OR_NODE_INTERFACE 1 /* outer boundary: interpolation node                */
#define OR_NODE_WALL 2      /* on the solid wall of the lamina                   */

/* error codes */
#define OR_OK 0
#define OR_E_ARG -1
#define OR_E_NOMEM -2
#define OR_E_STATE -5
#define OR_E_UNSTABLE -4

typedef struct or_config {
  int32_t nx, ny;   /* background lattice nodes                         */
  int32_t nux, nuy; /* body-fitted grid nodes (0,0: lattice only)       */
  double h_u;       /* grid spacing (lattice units)                     */
  double b;         /* lamina width L (0: no body)                      */
  double thickness; /* lamina thickness T (must equal h_u)              */
  double tau;       /* structured relaxation time tau_s                 */
  double kc;        /* Keulegan-Carpenter number 2 pi A / L             */
  double beta;      /* frequency parameter omega L^2 / (2 pi nu)        */
  int32_t n_sub;    /* sub-steps per structured step; 0: automatic      */
  int32_t bc;       /* OR_BC_*                                          */
  int32_t flags;    /* OR_FLAG_*                                        */
  int64_t max_steps;/* capacity of the force history                    */
} or_config;

/* grid without the lamina slot (b still sets A and omega); for invariance
 * checks of the moving-grid coupling */
#define OR_FLAG_NO_BODY 1
/* planted mistakes in the lattice-grid exchange, for tests that show the pins
 * of the interface detect them */
#define OR_FLAG_PLANT_S_FACTOR 2   /* Eq.(postcollision2_s) with 1 - 1/tau_s in place
                                      of 2 (tau_s - 1)/(2 tau_s - 1)              */
#define OR_FLAG_PLANT_NO_KNEQ 4    /* f^neq,s not rescaled by 1 - 1/(2 tau_s) in the
                                      interface donors and the type-1 refill      */
#define OR_FLAG_PLANT_SWAP_BILIN_Y 8  /* bilinear weights mirrored in y           */
#define OR_FLAG_PLANT_SWAP_BILIN_X 16 /* bilinear weights mirrored in x           */
#define OR_FLAG_PLANT_BARY 32      /* barycentric weights of the grid interpolation
                                      and the type-3 refill taken in a rotated
                                      vertex order                                */

typedef struct or_info {
  double nu, tau_u, dt_u, A, omega, period, u_max, mach, reynolds, eps;
  int32_t n_sub, nnode, ntri, n_interface, n_wall, n_wall_edges;
  int32_t beta_limit_ok; /* 1 if beta < 2.6 eps^-1.6 (Eq. betalimit) */
  int64_t step;
  double y;              /* current lamina offset y(t_k)             */
  int64_t n_type1, n_type2, n_type3; /* refill counts, summed over steps */
} or_info;

typedef struct or_sim or_sim;
typedef struct or_mesh or_mesh;

/* ---- equilibrium, Eq.(local_eq) ------------------------------------- */
void or_feq(double rho, double ux, double uy, double feq[9]);
void or_d2q9(int32_t cx[9], int32_t cy[9], double w[9]);

/* ---- structured lattice, Eq.(LBE) ------------------------------------ */
/* One pull stream + BGK collide from A (post-collision t) to B (post-collision
 * t+1) over an nx*ny lattice stored [9][ny][nx]. disc: per-node flag (NULL =
 * every node computes); non-computing nodes copy A to B. Walls (bc 0) may move
 * tangentially with x-velocities u_bot, u_top. */
void or_lattice_step(const double *A, double *B, int32_t nx, int32_t ny,
                     int32_t bc, double tau, double u_bot, double u_top,
                     const uint8_t *disc);

/* ---- finite-volume mesh, Eq.(ulbe) ----------------------------------- */
/* lamina grid: nux*nuy nodes, spacing h, lamina slot of width b (0: none) */
or_mesh *or_mesh_lamina(int32_t nux, int32_t nuy, double h, double b);
/* the lamina grid with graded spacing: columns at local x = X[i], rows at
 * y = Y[j] (strictly increasing), thickness Y[nuy/2] - Y[nuy/2-1] */
or_mesh *or_mesh_lamina_coords(int32_t nux, int32_t nuy, const double *X, const double *Y, double b);
/* doubly periodic nx*ny grid of spacing h, every node interior */
or_mesh *or_mesh_periodic(int32_t nx, int32_t ny, double h);
/* channel periodic in x, rows 0 and ny-1 are walls */
or_mesh *or_mesh_channel(int32_t nx, int32_t ny, double h);
void or_mesh_free(or_mesh *m);
int32_t or_mesh_nnode(const or_mesh *m);
int32_t or_mesh_ntri(const or_mesh *m);
int32_t or_mesh_kmax(const or_mesh *m);
/* node coordinates (local frame) and types */
void or_mesh_nodes(const or_mesh *m, double *x, double *y, int32_t *type);
/* triangles: [ntri][3] node ids and [ntri][3][2] vertex coordinates */
void or_mesh_triangles(const or_mesh *m, int32_t *tri, double *txy);
/* dense stencil export: nbr [nnode][kmax] (-1 padded, self first),
 * S [nnode][9][kmax], C [nnode][kmax], V [nnode] */
void or_mesh_stencil(const or_mesh *m, int32_t kmax, int32_t *nbr, double *S,
                     double *C, double *V);
/* point location: triangle containing (px,py) in the local frame, or -1;
 * lam gets the barycentric coordinates */
int32_t or_mesh_locate(const or_mesh *m, double px, double py, double lam[3]);
/* One sub-step of Eq.(ulbe) (interior / wall nodes) and Eq.(postcollision2_u)
 * (interface nodes). f, fout: [9][nnode]. star_eq / star_neq: [9][nnode],
 * read at interface nodes only (may be NULL when there are none). uwx, uwy:
 * per-node wall velocity, read at wall nodes only (may be NULL if no walls). */
void or_fv_substep(const or_mesh *m, const double *f, const double *star_eq,
                   const double *star_neq, double *fout, double tau_u,
                   double dt_u, const double *uwx, const double *uwy);
/* wall force: sum over wall edges, trapezoid rule; f [9][nnode] */
void or_mesh_force(const or_mesh *m, const double *f, double F[2]);

/* ---- the hybrid method ----------------------------------------------- */
int or_create(const or_config *cfg, or_sim **out);
/* host threads of the per-node loops (lattice stream-collide, grid
 * sub-steps), 1 by default; n <= 0 only queries. Results do not depend on
 * it. Returns the number in effect (always 1 in a build without OpenMP). */
int or_set_threads(int32_t n);
/* a case with a graded grid: columns at local x = X[nux], rows at y =
 * Y[nuy] (rows symmetric about the lamina, thickness Y[nuy/2] - Y[nuy/2-1]) */
int or_create_graded(const or_config *cfg, const double *X, const double *Y, or_sim **out);
/* a case on any triangulation of the grid region (Sec. Hybrid lattice
 * Boltzmann method: an unstructured mesh around the body): nodes at local
 * coordinates xy [nnode][2] (lamina centre at the origin), types [nnode]
 * (OR_NODE_*: the outer boundary's nodes are interface nodes, the lamina's
 * wall nodes), counter-clockwise triangles tri [ntri][3]. The grid's outer
 * boundary is the bounding box of the nodes (symmetric in y); the lamina is
 * |x| < b/2, |y| < thickness/2 (cfg->nux, nuy, h_u unused). */
int or_create_mesh(const or_config *cfg, int32_t nnode, const double *xy, const int32_t *type, int32_t ntri,
                   const int32_t *tri, or_sim **out);
/* a prescribed deformation of a case on a given triangulation (before the
 * first step): the lamina bends as Y(x, t) = A sin(omega t) +
 * B sin(omega t + phi) (2x/b)^2 and the grid follows it (see
 * hlbm_oracle.c); |B| < 1 */
int or_set_deformation(or_sim *s, double B, double phi);
void or_destroy(or_sim *s);
int or_step(or_sim *s, int64_t nsteps);
int or_info_get(const or_sim *s, or_info *out);
const or_mesh *or_sim_mesh(const or_sim *s);
/* lattice [9][ny][nx] (post-collision at t_k), mesh [9][nnode] at t_k */
int or_get_lattice(const or_sim *s, double *out);
int or_set_lattice(or_sim *s, const double *in);
int or_get_mesh(const or_sim *s, double *out);
int or_set_mesh(or_sim *s, const double *in);
/* force history: entry k holds (Fx, Fy) at t = k+1; returns count */
int64_t or_history(const or_sim *s, double *out, int64_t cap);
/* two-way coupled motion (before the first step): M y'' + C y' + K y = F_y
 * per unit depth, from (y0, v0), |y| <= y_max (see hlbm_oracle.c) */
int or_set_motion(or_sim *s, double M, double K, double C, double y0, double v0, double y_max);
/* (y, v) after each step of a coupled run: entry k at t = k+1 */
int64_t or_motion_history(const or_sim *s, double *out, int64_t cap);
/* status of lattice node (x,y) at step k: 0 disc, 1 interpolation, 2 unused */
int32_t or_lattice_status(const or_sim *s, int64_t k, int32_t x, int32_t y);
/* tangential x-velocities of the lattice's y walls (bc 0; both 0 unless set) */
int or_set_walls(or_sim *s, double u_bot, double u_top);
/* A case whose grid is a band on a wall instead of a lamina: the band is
 * periodic in x with cfg->nx columns and nband rows of unit spacing, node
 * (i, j) at lattice position (x_off + i, y_wall + j); row 0 lies on a wall
 * that moves tangentially with velocity U cos(omega t), the top row takes
 * Eq.(postcollision2_u) from the lattice, and lattice nodes below the band's
 * top row minus the margin of 2 are carried by the grid (the fictitious line
 * of Sec. Refill procedure becomes y = y_wall + nband - 3). The grid does not
 * move. Used by the Stokes-layer pin of the lattice-grid interface.
 * cfg: nx, ny, tau, n_sub, bc (must be OR_BC_PERIODIC_X_WALLS_Y), flags
 * (planted mistakes only), max_steps; the other fields are ignored. */
int or_create_wallband(const or_config *cfg, int32_t nband, double x_off, double y_wall, double U,
                       double omega, or_sim **out);
/* Probes of the two interpolations of the exchange, for tests. Both return
 * (rho, ux, uy, f^neq[9]) at a point given in lattice coordinates:
 * or_probe_bilinear over the four lattice nodes of the enclosing cell, from
 * the pre-collision populations at t_{k+1} (type-1 refill and interface
 * donors); or_probe_grid over the enclosing grid triangle at the current
 * offset (Eq.(postcollision2_s)). OR_E_STATE if no triangle holds the point. */
int or_probe_bilinear(const or_sim *s, double X, double Y, double out[12]);
int or_probe_grid(const or_sim *s, double X, double Y, double out[12]);

/* ---- structured refinement levels ------------------------------------ */
/* Level 0 is an nx0 x ny0 lattice with boundaries bc0 (walls may move with
 * x-velocities u_bot, u_top under bc 0). Level l+1 covers the node box
 * box[4l .. 4l+3] = (x0, y0, x1, y1) of level l (inclusive, at least two
 * nodes inside level l's edges, at least four cells wide) with twice the
 * resolution: 2 (x1 - x0) + 1 by 2 (y1 - y0) + 1 nodes. The finest level is
 * the hybrid case `fine` (bc OR_BC_RING, nx and ny as implied by the last
 * box, tau and the body in its own lattice units); tau of each coarser level
 * follows from equal viscosity. One or_ml_step advances level 0 by one step
 * and level l by 2^l steps. */
#define OR_ML_MAX_LEVELS 8
/* planted mistakes, for tests that show the pins detect them */
#define OR_ML_FLAG_PLANT_NO_RESCALE 256 /* f^neq not rescaled between levels */
#define OR_ML_FLAG_PLANT_SAME_TAU 512   /* every level relaxes with the finest tau */
typedef struct or_ml or_ml;
int or_ml_create(const or_config *fine, int32_t nlevels, int32_t nx0, int32_t ny0, int32_t bc0,
                 double u_bot, double u_top, const int32_t *box, int32_t flags, or_ml **out);
void or_ml_destroy(or_ml *s);
int or_ml_step(or_ml *s, int64_t nsteps);
int or_ml_level_shape(const or_ml *s, int32_t level, int32_t *nx, int32_t *ny, double *tau);
/* level state [9][ny][nx], post-collision at the current time */
int or_ml_get_level(const or_ml *s, int32_t level, double *out);
int or_ml_set_level(or_ml *s, int32_t level, const double *in);
/* the finest level's hybrid case (history, grid, info) */
or_sim *or_ml_finest(or_ml *s);
int64_t or_ml_steps(const or_ml *s);

/* ---- hydrodynamic function fit (Sec. Hydrodynamic function extraction) -- */
/* hist: (Fx,Fy) pairs, entry k at t=k+1. Window [t0, t1) in periods.
 * Returns 0 and theta = (Re, Im), or OR_E_ARG if the window holds < 2 samples. */
int or_fit_theta(const double *hist, int64_t n, double omega, double A,
                 double b, double t0, double t1, double theta[2]);

#ifdef __cplusplus
}
#endif
#endif
