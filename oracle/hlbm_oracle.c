/*
 * hlbm_oracle.c -- plain FP64 CPU oracle of the moving-grid hybrid lattice
 * Boltzmann method (MG-HLBM), Di Ilio et al., arXiv 2006.13631.
 *
 * TEST INFRASTRUCTURE ONLY: see hlbm_oracle.h. Nothing here is tuned; every
 * function is a direct, loop-by-loop statement of the passage it cites.
 *
 * Units: lattice spacing and structured time step are 1 (Delta x_s = Delta
 * t_s = 1), reference density 1. D2Q9 with c_s^2 = 1/3 (Sec. 3, below
 * Eq.(ulbe)); the paper does not print the weights, the standard D2Q9 set is
 * used.
 */
#include "hlbm_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Scalar of every quantity that depends on the physical parameters. The
 * default build uses double. Built with -DOR_COMPLEX_STEP it uses
 * double _Complex: A, omega and tau can then carry an imaginary perturbation
 * i h, and Im(output)/h is the exact derivative of the discrete method
 * (complex-step differentiation; every decision uses the real part). The
 * grid geometry and its matrices stay double. */
#ifdef OR_COMPLEX_STEP
#include <complex.h>
typedef double _Complex real;
#define RE(x) creal(x)
#define RSIN csin
#define RCOS ccos
#else
typedef double real;
#define RE(x) (x)
#define RSIN sin
#define RCOS cos
#endif

/* ------------------------------------------------------------------ */
/* D2Q9 velocity set: rest, 4 axis, 4 diagonal directions              */
/* ------------------------------------------------------------------ */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double CS2 = 1.0 / 3.0; /* lattice speed of sound squared */

/* host threads of the per-node loops; 1 (serial) unless or_set_threads asks */
static int or_threads = 1;

void or_d2q9(int32_t cx[9], int32_t cy[9], double w[9]) {
  for (int i = 0; i < 9; ++i) {
    cx[i] = CX[i];
    cy[i] = CY[i];
    w[i] = WT[i];
  }
}

/* Eq.(local_eq): second-order polynomial equilibrium. */
static void feq_r(real rho, real ux, real uy, real feq[9]) {
  const real uu = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) {
    const real cu = CX[i] * ux + CY[i] * uy;
    feq[i] = WT[i] * rho *
             (1.0 + cu / CS2 + (cu * cu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

#ifndef OR_COMPLEX_STEP
void or_feq(double rho, double ux, double uy, double feq[9]) { feq_r(rho, ux, uy, feq); }
#endif

/* density and velocity: the first two moments of f (text after Eq.(local_eq)) */
static void moments(const real f[9], real *rho, real *ux, real *uy) {
  real r = 0.0, mx = 0.0, my = 0.0;
  for (int i = 0; i < 9; ++i) {
    r += f[i];
    mx += CX[i] * f[i];
    my += CY[i] * f[i];
  }
  *rho = r;
  *ux = mx / r;
  *uy = my / r;
}

/* ------------------------------------------------------------------ */
/* Structured lattice, Eq.(LBE)                                        */
/* ------------------------------------------------------------------ */
static size_t lidx(int nx, int ny, int q, int x, int y) {
  return ((size_t)q * (size_t)ny + (size_t)y) * (size_t)nx + (size_t)x;
}

static int wrap(int a, int n) { return ((a % n) + n) % n; }

/* Streaming (left side of Eq.(LBE)) written in pull form: the population
 * arriving at (x,y) along c_i left x - c_i one step earlier. Across a y wall
 * (bc 0) it is the opposite population of the same node, reflected halfway;
 * a wall moving with x-velocity uw adds 2 w_i rho0 c_i.u_w / c_s^2.
 * The paper's boundaries (bc 2): across an x wall (at rest) the same
 * halfway reflection; at a y end, where no population arrives from outside,
 * the incoming one equals that of the next row in (zero normal gradient),
 * which that node pulled from this node's own row. A population crossing
 * both a wall and an end (corner nodes) is reflected by the wall.
 * A ring-fed level (bc 3) pulls only at nodes off its outermost ring, whose
 * neighbours all lie inside the lattice. */
static void pull_node(const real *A, int nx, int ny, int bc, int x, int y,
                      real u_bot, real u_top, real f[9]) {
  for (int i = 0; i < 9; ++i) {
    if (bc == OR_BC_RING) {
      f[i] = A[lidx(nx, ny, i, x - CX[i], y - CY[i])];
      continue;
    }
    if (bc == OR_BC_PAPER) {
      const int xp = x - CX[i];
      if (xp < 0 || xp >= nx) {
        f[i] = A[lidx(nx, ny, OPP[i], x, y)];
        continue;
      }
      int yp = y - CY[i];
      if (yp < 0 || yp >= ny) yp = y;
      f[i] = A[lidx(nx, ny, i, xp, yp)];
      continue;
    }
    const int xs = wrap(x - CX[i], nx);
    int ys = y - CY[i];
    if (bc == OR_BC_PERIODIC) {
      ys = wrap(ys, ny);
    } else if (ys < 0 || ys >= ny) {
      const real uw = (ys < 0) ? u_bot : u_top;
      f[i] = A[lidx(nx, ny, OPP[i], x, y)] + 2.0 * WT[i] * 1.0 * (CX[i] * uw) / CS2;
      continue;
    }
    f[i] = A[lidx(nx, ny, i, xs, ys)];
  }
}

static void lattice_step_r(const real *A, real *B, int32_t nx, int32_t ny,
                           int32_t bc, real tau, real u_bot, real u_top,
                           const uint8_t *disc) {
  /* nodes are independent: rows may run on several threads (same results) */
#pragma omp parallel for schedule(static) num_threads(or_threads) if (or_threads > 1)
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      /* the ring of a ring-fed level is written from the coarser level */
      if (bc == OR_BC_RING && (x == 0 || y == 0 || x == nx - 1 || y == ny - 1)) continue;
      if (disc && !disc[(size_t)y * nx + x]) {
        for (int i = 0; i < 9; ++i) B[lidx(nx, ny, i, x, y)] = A[lidx(nx, ny, i, x, y)];
        continue;
      }
      real f[9], feq[9], rho, ux, uy;
      pull_node(A, nx, ny, bc, x, y, u_bot, u_top, f);
      moments(f, &rho, &ux, &uy);
      feq_r(rho, ux, uy, feq);
      /* Eq.(LBE) with Delta t_s = 1: relax toward equilibrium */
      for (int i = 0; i < 9; ++i)
        B[lidx(nx, ny, i, x, y)] = f[i] - (1.0 / tau) * (f[i] - feq[i]);
    }
  }
}

#ifndef OR_COMPLEX_STEP
void or_lattice_step(const double *A, double *B, int32_t nx, int32_t ny,
                     int32_t bc, double tau, double u_bot, double u_top,
                     const uint8_t *disc) {
  lattice_step_r(A, B, nx, ny, bc, tau, u_bot, u_top, disc);
}
#endif

/* ------------------------------------------------------------------ */
/* Triangular body-fitted grid and its finite-volume matrices          */
/* ------------------------------------------------------------------ */
#define KCAP 16 /* neighbour slots per node (self included) */

struct or_mesh {
  int nnode, ntri;
  double *x, *y; /* node coordinates, local frame */
  int *type;     /* OR_NODE_* */
  int *tri;      /* [ntri][3] */
  double *txy;   /* [ntri][3][2] vertex coordinates (unwrapped) */
  /* stencil: per node up to KCAP neighbours, slot 0 = the node itself */
  int *nk;       /* [nnode] */
  int *nbr;      /* [nnode][KCAP] */
  double *S;     /* [nnode][9][KCAP] streaming matrix S_ik */
  double *C;     /* [nnode][KCAP] collision matrix C_ik */
  double *V;     /* [nnode] control-volume area */
  /* wall edges (force) */
  int nwe;
  int *we;       /* [nwe][2] */
  double *wn;    /* [nwe][2] unit normal pointing out of the body */
  double *wl;    /* [nwe] length */
  /* bucket grid for point location */
  double bx0, by0, bh;
  int bnx, bny;
  int *bstart, *blist;
  /* lamina geometry (local frame) */
  double b, T;
};

static void *xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

void or_mesh_free(or_mesh *m) {
  if (!m) return;
  free(m->x); free(m->y); free(m->type); free(m->tri); free(m->txy);
  free(m->nk); free(m->nbr); free(m->S); free(m->C); free(m->V);
  free(m->we); free(m->wn); free(m->wl); free(m->bstart); free(m->blist);
  free(m);
}

int32_t or_mesh_nnode(const or_mesh *m) { return m->nnode; }
int32_t or_mesh_ntri(const or_mesh *m) { return m->ntri; }
int32_t or_mesh_kmax(const or_mesh *m) {
  int k = 0;
  for (int p = 0; p < m->nnode; ++p)
    if (m->nk[p] > k) k = m->nk[p];
  return k;
}

void or_mesh_nodes(const or_mesh *m, double *x, double *y, int32_t *type) {
  for (int p = 0; p < m->nnode; ++p) {
    if (x) x[p] = m->x[p];
    if (y) y[p] = m->y[p];
    if (type) type[p] = m->type[p];
  }
}

void or_mesh_triangles(const or_mesh *m, int32_t *tri, double *txy) {
  for (int t = 0; t < m->ntri; ++t)
    for (int a = 0; a < 3; ++a) {
      if (tri) tri[3 * t + a] = m->tri[3 * t + a];
      if (txy) {
        txy[6 * t + 2 * a] = m->txy[6 * t + 2 * a];
        txy[6 * t + 2 * a + 1] = m->txy[6 * t + 2 * a + 1];
      }
    }
}

/* barycentric coordinates of (px,py) in the triangle with vertices v[3][2] */
static void bary(const double *v, double px, double py, double lam[3]) {
  const double x0 = v[0], y0 = v[1], x1 = v[2], y1 = v[3], x2 = v[4], y2 = v[5];
  const double d = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0);
  lam[1] = ((px - x0) * (y2 - y0) - (x2 - x0) * (py - y0)) / d;
  lam[2] = ((x1 - x0) * (py - y0) - (px - x0) * (y1 - y0)) / d;
  lam[0] = 1.0 - lam[1] - lam[2];
}

/* same, for a point whose coordinates may carry a perturbation */
static void bary_r(const double *v, real px, real py, real lam[3]) {
  const double x0 = v[0], y0 = v[1], x1 = v[2], y1 = v[3], x2 = v[4], y2 = v[5];
  const double d = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0);
  lam[1] = ((px - x0) * (y2 - y0) - (x2 - x0) * (py - y0)) / d;
  lam[2] = ((x1 - x0) * (py - y0) - (px - x0) * (y1 - y0)) / d;
  lam[0] = 1.0 - lam[1] - lam[2];
}

typedef struct { int lo, hi, slot; } edge_t;

static int edge_cmp(const void *x, const void *y) {
  const edge_t *a = (const edge_t *)x, *b = (const edge_t *)y;
  if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
  if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;
  return a->slot < b->slot ? -1 : (a->slot > b->slot);
}

static int slot_of(or_mesh *m, int p, int q) {
  for (int k = 0; k < m->nk[p]; ++k)
    if (m->nbr[p * KCAP + k] == q) return k;
  return -1;
}

static int add_nbr(or_mesh *m, int p, int q) {
  int s = slot_of(m, p, q);
  if (s >= 0) return s;
  if (m->nk[p] >= KCAP) return -1;
  m->nbr[p * KCAP + m->nk[p]] = q;
  return m->nk[p]++;
}

/* Median-dual control volume of each node (centroids joined to edge
 * midpoints; closed by half-edges where the grid ends), f linear on each
 * triangle. Reading of S_ik and C_ik, which the paper cites but does not give
 * (Sec. 3, after Eq.(ulbe)):
 *   S_ik = -(1/V_P) * (coefficient of f(P_k) in the outflow of population i
 *           through the boundary of the control volume of P),
 *   C_ik =  (1/V_P) * integral over the control volume of the linear shape
 *           function of P_k.
 * Both integrals are exact for piecewise-linear f. */
static int assemble(or_mesh *m) {
  const int N = m->nnode;
  m->nk = xcalloc(N, sizeof(int));
  m->nbr = xcalloc((size_t)N * KCAP, sizeof(int));
  m->S = xcalloc((size_t)N * 9 * KCAP, sizeof(double));
  m->C = xcalloc((size_t)N * KCAP, sizeof(double));
  m->V = xcalloc(N, sizeof(double));
  if (!m->nk || !m->nbr || !m->S || !m->C || !m->V) return OR_E_NOMEM;
  for (int p = 0; p < N; ++p) {
    for (int k = 0; k < KCAP; ++k) m->nbr[p * KCAP + k] = -1;
    add_nbr(m, p, p); /* slot 0: the pivotal node itself (k = 0 in Eq.(ulbe)) */
  }
  for (int t = 0; t < m->ntri; ++t)
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c)
        if (add_nbr(m, m->tri[3 * t + a], m->tri[3 * t + c]) < 0) return OR_E_ARG;

  double *Sacc = m->S, *Cacc = m->C;
  for (int t = 0; t < m->ntri; ++t) {
    const int *v = &m->tri[3 * t];
    const double *p = &m->txy[6 * t];
    const double area = 0.5 * ((p[2] - p[0]) * (p[5] - p[1]) - (p[4] - p[0]) * (p[3] - p[1]));
    if (!(area > 0.0)) return OR_E_ARG;
    const double gx = (p[0] + p[2] + p[4]) / 3.0, gy = (p[1] + p[3] + p[5]) / 3.0;
    for (int a = 0; a < 3; ++a) m->V[v[a]] += area / 3.0;

    /* collision matrix: integrate each shape function over the part of the
     * control volume of vertex a inside this triangle, the quadrilateral
     * (a, mid(a,b), centroid, mid(a,c)), split into two triangles. A linear
     * function integrates to area * mean of its vertex values. */
    for (int a = 0; a < 3; ++a) {
      const int b = (a + 1) % 3, c = (a + 2) % 3;
      const double ax = p[2 * a], ay = p[2 * a + 1];
      const double mbx = 0.5 * (ax + p[2 * b]), mby = 0.5 * (ay + p[2 * b + 1]);
      const double mcx = 0.5 * (ax + p[2 * c]), mcy = 0.5 * (ay + p[2 * c + 1]);
      const double sub[2][6] = {{ax, ay, mbx, mby, gx, gy}, {ax, ay, gx, gy, mcx, mcy}};
      for (int s = 0; s < 2; ++s) {
        const double *q = sub[s];
        const double sa = 0.5 * fabs((q[2] - q[0]) * (q[5] - q[1]) - (q[4] - q[0]) * (q[3] - q[1]));
        double lsum[3] = {0.0, 0.0, 0.0};
        for (int r = 0; r < 3; ++r) {
          double lam[3];
          bary(p, q[2 * r], q[2 * r + 1], lam);
          for (int j = 0; j < 3; ++j) lsum[j] += lam[j];
        }
        for (int j = 0; j < 3; ++j)
          Cacc[v[a] * KCAP + slot_of(m, v[a], v[j])] += sa * lsum[j] / 3.0;
      }
    }

    /* streaming matrix, interior faces: the face between the control volumes
     * of vertices a and b inside this triangle runs from mid(a,b) to the
     * centroid. Outflow of population i from the volume of a through it is
     * (c_i . n) * length * f(face midpoint), n pointing from a toward b. */
    for (int a = 0; a < 3; ++a) {
      const int b = (a + 1) % 3;
      const double mx = 0.5 * (p[2 * a] + p[2 * b]), my = 0.5 * (p[2 * a + 1] + p[2 * b + 1]);
      double nlx = gy - my, nly = -(gx - mx); /* normal scaled by face length */
      if (nlx * (p[2 * b] - p[2 * a]) + nly * (p[2 * b + 1] - p[2 * a + 1]) < 0.0) {
        nlx = -nlx;
        nly = -nly;
      }
      double lam[3];
      bary(p, 0.5 * (mx + gx), 0.5 * (my + gy), lam);
      for (int i = 0; i < 9; ++i) {
        const double cn = CX[i] * nlx + CY[i] * nly;
        for (int j = 0; j < 3; ++j) {
          Sacc[((size_t)v[a] * 9 + i) * KCAP + slot_of(m, v[a], v[j])] -= cn * lam[j];
          Sacc[((size_t)v[b] * 9 + i) * KCAP + slot_of(m, v[b], v[j])] += cn * lam[j];
        }
      }
    }
  }

  /* boundary faces: an edge that belongs to one triangle only ends the grid.
   * Each of its end nodes closes its control volume with the half of the edge
   * next to it; f along it is linear between the two end nodes. */
  int nwe = 0;
  int *edge_count = xcalloc((size_t)m->ntri * 3, sizeof(int));
  edge_t *edges = xcalloc((size_t)m->ntri * 3, sizeof(edge_t));
  if (!edge_count || !edges) return OR_E_NOMEM;
  for (int t = 0; t < m->ntri; ++t)
    for (int e = 0; e < 3; ++e) {
      const int a = m->tri[3 * t + e], b = m->tri[3 * t + (e + 1) % 3];
      edge_t *E = &edges[3 * t + e];
      E->lo = a < b ? a : b;
      E->hi = a < b ? b : a;
      E->slot = 3 * t + e;
    }
  qsort(edges, (size_t)m->ntri * 3, sizeof(edge_t), edge_cmp);
  for (size_t r = 0; r < (size_t)m->ntri * 3;) {
    size_t q = r;
    while (q < (size_t)m->ntri * 3 && edges[q].lo == edges[r].lo && edges[q].hi == edges[r].hi) ++q;
    for (size_t u = r; u < q; ++u) edge_count[edges[u].slot] = (int)(q - r - 1);
    r = q;
  }
  free(edges);
  for (int t = 0; t < m->ntri; ++t)
    for (int e = 0; e < 3; ++e) {
      const int a = m->tri[3 * t + e], b = m->tri[3 * t + (e + 1) % 3];
      if (edge_count[3 * t + e] == 0 && m->type[a] == OR_NODE_WALL && m->type[b] == OR_NODE_WALL) ++nwe;
    }
  m->nwe = nwe;
  m->we = xcalloc((size_t)2 * nwe, sizeof(int));
  m->wn = xcalloc((size_t)2 * nwe, sizeof(double));
  m->wl = xcalloc(nwe, sizeof(double));
  int w = 0;
  for (int t = 0; t < m->ntri; ++t) {
    const double *p = &m->txy[6 * t];
    for (int e = 0; e < 3; ++e) {
      if (edge_count[3 * t + e] != 0) continue;
      const int ea = e, eb = (e + 1) % 3, ec = (e + 2) % 3;
      const int a = m->tri[3 * t + ea], b = m->tri[3 * t + eb];
      const double ex = p[2 * eb] - p[2 * ea], ey = p[2 * eb + 1] - p[2 * ea + 1];
      double nlx = ey, nly = -ex; /* outward normal of the grid, scaled by length */
      if (nlx * (p[2 * ec] - p[2 * ea]) + nly * (p[2 * ec + 1] - p[2 * ea + 1]) > 0.0) {
        nlx = -nlx;
        nly = -nly;
      }
      const int ends[2] = {ea, eb};
      for (int s = 0; s < 2; ++s) {
        const int me = ends[s], other = ends[1 - s];
        const int node = m->tri[3 * t + me];
        /* half edge from this end to the edge midpoint; its midpoint sits at
         * 3/4 of the way from the other end */
        double lam[3];
        bary(p, 0.75 * p[2 * me] + 0.25 * p[2 * other], 0.75 * p[2 * me + 1] + 0.25 * p[2 * other + 1], lam);
        for (int i = 0; i < 9; ++i) {
          const double cn = 0.5 * (CX[i] * nlx + CY[i] * nly);
          for (int j = 0; j < 3; ++j)
            Sacc[((size_t)node * 9 + i) * KCAP + slot_of(m, node, m->tri[3 * t + j])] -= cn * lam[j];
        }
      }
      if (m->type[a] == OR_NODE_WALL && m->type[b] == OR_NODE_WALL) {
        const double len = sqrt(ex * ex + ey * ey);
        m->we[2 * w] = a;
        m->we[2 * w + 1] = b;
        m->wn[2 * w] = -nlx / len; /* the body lies outside the grid */
        m->wn[2 * w + 1] = -nly / len;
        m->wl[w] = len;
        ++w;
      }
    }
  }
  free(edge_count);

  for (int p = 0; p < N; ++p) {
    if (!(m->V[p] > 0.0)) return OR_E_ARG;
    for (int k = 0; k < m->nk[p]; ++k) {
      m->C[p * KCAP + k] /= m->V[p];
      for (int i = 0; i < 9; ++i) m->S[((size_t)p * 9 + i) * KCAP + k] /= m->V[p];
    }
  }
  return OR_OK;
}

/* bucket grid: each triangle is listed in every unit bucket its bounding box
 * touches, in increasing triangle order */
static int build_buckets(or_mesh *m) {
  double x0 = 1e300, y0 = 1e300, x1 = -1e300, y1 = -1e300;
  for (int t = 0; t < m->ntri; ++t)
    for (int a = 0; a < 3; ++a) {
      const double px = m->txy[6 * t + 2 * a], py = m->txy[6 * t + 2 * a + 1];
      if (px < x0) x0 = px;
      if (px > x1) x1 = px;
      if (py < y0) y0 = py;
      if (py > y1) y1 = py;
    }
  m->bh = 1.0;
  m->bx0 = x0;
  m->by0 = y0;
  m->bnx = (int)floor((x1 - x0) / m->bh) + 1;
  m->bny = (int)floor((y1 - y0) / m->bh) + 1;
  const size_t nb = (size_t)m->bnx * m->bny;
  int *count = xcalloc(nb + 1, sizeof(int));
  m->bstart = xcalloc(nb + 1, sizeof(int));
  if (!count || !m->bstart) return OR_E_NOMEM;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      m->bstart[0] = 0;
      for (size_t i = 0; i < nb; ++i) m->bstart[i + 1] = m->bstart[i] + count[i];
      m->blist = xcalloc((size_t)m->bstart[nb], sizeof(int));
      if (!m->blist) return OR_E_NOMEM;
      memset(count, 0, nb * sizeof(int));
    }
    for (int t = 0; t < m->ntri; ++t) {
      double tx0 = 1e300, ty0 = 1e300, tx1 = -1e300, ty1 = -1e300;
      for (int a = 0; a < 3; ++a) {
        const double px = m->txy[6 * t + 2 * a], py = m->txy[6 * t + 2 * a + 1];
        if (px < tx0) tx0 = px;
        if (px > tx1) tx1 = px;
        if (py < ty0) ty0 = py;
        if (py > ty1) ty1 = py;
      }
      int i0 = (int)floor((tx0 - m->bx0) / m->bh) - 1, i1 = (int)floor((tx1 - m->bx0) / m->bh) + 1;
      int j0 = (int)floor((ty0 - m->by0) / m->bh) - 1, j1 = (int)floor((ty1 - m->by0) / m->bh) + 1;
      if (i0 < 0) i0 = 0;
      if (j0 < 0) j0 = 0;
      if (i1 >= m->bnx) i1 = m->bnx - 1;
      if (j1 >= m->bny) j1 = m->bny - 1;
      for (int j = j0; j <= j1; ++j)
        for (int i = i0; i <= i1; ++i) {
          const size_t bi = (size_t)j * m->bnx + i;
          if (pass == 1) m->blist[m->bstart[bi] + count[bi]] = t;
          ++count[bi];
        }
    }
  }
  free(count);
  return OR_OK;
}

/* Point location with a closed inside test; a point on a shared edge goes to
 * the lowest-numbered triangle (triangles are numbered by cell, row-major,
 * lower triangle first). Interpolation is continuous, so the choice only
 * changes rounding. */
int32_t or_mesh_locate(const or_mesh *m, double px, double py, double lam[3]) {
  const double tol = 1e-12;
  const int bi = (int)floor((px - m->bx0) / m->bh), bj = (int)floor((py - m->by0) / m->bh);
  if (bi < 0 || bj < 0 || bi >= m->bnx || bj >= m->bny) return -1;
  const size_t b = (size_t)bj * m->bnx + bi;
  for (int s = m->bstart[b]; s < m->bstart[b + 1]; ++s) {
    const int t = m->blist[s];
    double l[3];
    bary(&m->txy[6 * t], px, py, l);
    if (l[0] >= -tol && l[1] >= -tol && l[2] >= -tol) {
      lam[0] = l[0];
      lam[1] = l[1];
      lam[2] = l[2];
      return t;
    }
  }
  return -1;
}

/* quad split into two triangles; the diagonal direction is mirrored about the
 * vertical centre line of the grid so the grid is left-right symmetric */
static void add_cell(or_mesh *m, int *nt, int n00, int n10, int n01, int n11,
                     double x0, double y0, double h, int diag_up) {
  const double X[4] = {x0, x0 + h, x0, x0 + h}, Y[4] = {y0, y0, y0 + h, y0 + h};
  const int id[4] = {n00, n10, n01, n11};
  int tris[2][3];
  if (diag_up) { /* diagonal from (0,0) to (1,1) */
    tris[0][0] = 0; tris[0][1] = 1; tris[0][2] = 3;
    tris[1][0] = 0; tris[1][1] = 3; tris[1][2] = 2;
  } else { /* diagonal from (1,0) to (0,1) */
    tris[0][0] = 0; tris[0][1] = 1; tris[0][2] = 2;
    tris[1][0] = 1; tris[1][1] = 3; tris[1][2] = 2;
  }
  for (int s = 0; s < 2; ++s) {
    for (int a = 0; a < 3; ++a) {
      m->tri[3 * (*nt) + a] = id[tris[s][a]];
      m->txy[6 * (*nt) + 2 * a] = X[tris[s][a]];
      m->txy[6 * (*nt) + 2 * a + 1] = Y[tris[s][a]];
    }
    ++(*nt);
  }
}

static or_mesh *mesh_alloc(int nnode, int maxtri) {
  or_mesh *m = xcalloc(1, sizeof(or_mesh));
  if (!m) return NULL;
  m->nnode = nnode;
  m->x = xcalloc(nnode, sizeof(double));
  m->y = xcalloc(nnode, sizeof(double));
  m->type = xcalloc(nnode, sizeof(int));
  m->tri = xcalloc((size_t)3 * maxtri, sizeof(int));
  m->txy = xcalloc((size_t)6 * maxtri, sizeof(double));
  if (!m->x || !m->y || !m->type || !m->tri || !m->txy) {
    or_mesh_free(m);
    return NULL;
  }
  return m;
}

static or_mesh *mesh_finish(or_mesh *m) {
  if (assemble(m) != OR_OK || build_buckets(m) != OR_OK) {
    or_mesh_free(m);
    return NULL;
  }
  return m;
}

/* Body-fitted grid around the lamina: nux*nuy nodes with spacing h; node
 * (i,j) at local x = (i - nux/2) h, y = (j - (nuy-1)/2) h (lamina centre at
 * the origin). The lamina, of width b and thickness h, fills the slot between
 * rows nuy/2-1 and nuy/2 for |x| <= b/2; those cells are not meshed. Nodes on
 * the slot boundary are wall nodes, nodes on the outer boundary are
 * interpolation nodes (Sec. Refill procedure), the rest discretization. */
or_mesh *or_mesh_lamina(int32_t nux, int32_t nuy, double h, double b) {
  if (nux < 4 || nuy < 4 || (nuy % 2) != 0 || !(h > 0.0) || b < 0.0) return NULL;
  or_mesh *m = mesh_alloc(nux * nuy, 2 * (nux - 1) * (nuy - 1));
  if (!m) return NULL;
  m->b = b;
  m->T = (b > 0.0) ? h : 0.0;
  const double half = 0.5 * b + 1e-9 * h;
  for (int j = 0; j < nuy; ++j)
    for (int i = 0; i < nux; ++i) {
      const int p = j * nux + i;
      m->x[p] = (double)(i - nux / 2) * h;
      m->y[p] = ((double)j - 0.5 * (double)(nuy - 1)) * h;
      if (b > 0.0 && (j == nuy / 2 - 1 || j == nuy / 2) && fabs(m->x[p]) <= half)
        m->type[p] = OR_NODE_WALL;
      else if (i == 0 || j == 0 || i == nux - 1 || j == nuy - 1)
        m->type[p] = OR_NODE_INTERFACE;
      else
        m->type[p] = OR_NODE_INTERIOR;
    }
  int nt = 0;
  for (int cj = 0; cj < nuy - 1; ++cj)
    for (int ci = 0; ci < nux - 1; ++ci) {
      const double x0 = (double)(ci - nux / 2) * h, y0 = ((double)cj - 0.5 * (double)(nuy - 1)) * h;
      if (b > 0.0 && cj == nuy / 2 - 1 && x0 >= -half && x0 + h <= half) continue; /* inside the lamina */
      const int n00 = cj * nux + ci;
      add_cell(m, &nt, n00, n00 + 1, n00 + nux, n00 + nux + 1, x0, y0, h, (x0 + 0.5 * h) < 0.0);
    }
  m->ntri = nt;
  return mesh_finish(m);
}

/* The same grid with graded spacing: column i at local x = X[i], row j at
 * local y = Y[j] (both strictly increasing); each cell is cut along the
 * diagonal of its side of the centre (the rising one for cells with
 * 2 ci + 1 < nux, as in the uniform grid), the lamina slot is the cells of
 * row nuy/2-1 inside |x| <= b/2, and the lamina thickness is
 * Y[nuy/2] - Y[nuy/2-1]. */
or_mesh *or_mesh_lamina_coords(int32_t nux, int32_t nuy, const double *X, const double *Y, double b) {
  if (nux < 4 || nuy < 4 || (nuy % 2) != 0 || !X || !Y || b < 0.0) return NULL;
  for (int i = 0; i + 1 < nux; ++i)
    if (!(X[i + 1] > X[i])) return NULL;
  for (int j = 0; j + 1 < nuy; ++j)
    if (!(Y[j + 1] > Y[j])) return NULL;
  or_mesh *m = mesh_alloc(nux * nuy, 2 * (nux - 1) * (nuy - 1));
  if (!m) return NULL;
  const double T = Y[nuy / 2] - Y[nuy / 2 - 1];
  m->b = b;
  m->T = (b > 0.0) ? T : 0.0;
  const double half = 0.5 * b + 1e-9 * T;
  for (int j = 0; j < nuy; ++j)
    for (int i = 0; i < nux; ++i) {
      const int p = j * nux + i;
      m->x[p] = X[i];
      m->y[p] = Y[j];
      if (b > 0.0 && (j == nuy / 2 - 1 || j == nuy / 2) && fabs(X[i]) <= half)
        m->type[p] = OR_NODE_WALL;
      else if (i == 0 || j == 0 || i == nux - 1 || j == nuy - 1)
        m->type[p] = OR_NODE_INTERFACE;
      else
        m->type[p] = OR_NODE_INTERIOR;
    }
  int nt = 0;
  for (int cj = 0; cj < nuy - 1; ++cj)
    for (int ci = 0; ci < nux - 1; ++ci) {
      if (b > 0.0 && cj == nuy / 2 - 1 && X[ci] >= -half && X[ci + 1] <= half) continue; /* inside the lamina */
      const int n00 = cj * nux + ci, n10 = n00 + 1, n01 = n00 + nux, n11 = n01 + 1;
      const double cx[4] = {X[ci], X[ci + 1], X[ci], X[ci + 1]}, cy[4] = {Y[cj], Y[cj], Y[cj + 1], Y[cj + 1]};
      const int id[4] = {n00, n10, n01, n11};
      static const int up[2][3] = {{0, 1, 3}, {0, 3, 2}}, down[2][3] = {{0, 1, 2}, {1, 3, 2}};
      const int(*tr)[3] = (2 * ci + 1 < nux) ? up : down;
      for (int t = 0; t < 2; ++t, ++nt)
        for (int a = 0; a < 3; ++a) {
          m->tri[3 * nt + a] = id[tr[t][a]];
          m->txy[6 * nt + 2 * a] = cx[tr[t][a]];
          m->txy[6 * nt + 2 * a + 1] = cy[tr[t][a]];
        }
    }
  m->ntri = nt;
  return mesh_finish(m);
}

or_mesh *or_mesh_periodic(int32_t nx, int32_t ny, double h) {
  if (nx < 3 || ny < 3 || !(h > 0.0)) return NULL;
  or_mesh *m = mesh_alloc(nx * ny, 2 * nx * ny);
  if (!m) return NULL;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      m->x[j * nx + i] = i * h;
      m->y[j * nx + i] = j * h;
      m->type[j * nx + i] = OR_NODE_INTERIOR;
    }
  int nt = 0;
  for (int cj = 0; cj < ny; ++cj)
    for (int ci = 0; ci < nx; ++ci) {
      const int i1 = (ci + 1) % nx, j1 = (cj + 1) % ny;
      add_cell(m, &nt, cj * nx + ci, cj * nx + i1, j1 * nx + ci, j1 * nx + i1, ci * h, cj * h, h,
               (ci + 0.5) < 0.5 * nx);
    }
  m->ntri = nt;
  return mesh_finish(m);
}

/* grid periodic in x, node (i, j) at (i h, j h); row 0 is a wall, the top
 * row a wall (a channel) or the outer boundary (a band on a wall) */
static or_mesh *mesh_strip(int32_t nx, int32_t ny, double h, int top_type) {
  if (nx < 3 || ny < 3 || !(h > 0.0)) return NULL;
  or_mesh *m = mesh_alloc(nx * ny, 2 * nx * (ny - 1));
  if (!m) return NULL;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      m->x[j * nx + i] = i * h;
      m->y[j * nx + i] = j * h;
      m->type[j * nx + i] = (j == 0) ? OR_NODE_WALL : (j == ny - 1) ? top_type : OR_NODE_INTERIOR;
    }
  int nt = 0;
  for (int cj = 0; cj < ny - 1; ++cj)
    for (int ci = 0; ci < nx; ++ci) {
      const int i1 = (ci + 1) % nx;
      add_cell(m, &nt, cj * nx + ci, cj * nx + i1, (cj + 1) * nx + ci, (cj + 1) * nx + i1, ci * h,
               cj * h, h, (ci + 0.5) < 0.5 * nx);
    }
  m->ntri = nt;
  return mesh_finish(m);
}

or_mesh *or_mesh_channel(int32_t nx, int32_t ny, double h) { return mesh_strip(nx, ny, h, OR_NODE_WALL); }

void or_mesh_stencil(const or_mesh *m, int32_t kmax, int32_t *nbr, double *S,
                     double *C, double *V) {
  for (int p = 0; p < m->nnode; ++p) {
    for (int k = 0; k < kmax; ++k) {
      const int in = k < m->nk[p] && k < KCAP;
      if (nbr) nbr[p * kmax + k] = in ? m->nbr[p * KCAP + k] : -1;
      if (C) C[p * kmax + k] = in ? m->C[p * KCAP + k] : 0.0;
      for (int i = 0; i < 9; ++i)
        if (S) S[((size_t)p * 9 + i) * kmax + k] = in ? m->S[((size_t)p * 9 + i) * KCAP + k] : 0.0;
    }
    if (V) V[p] = m->V[p];
  }
}

/* Eq.(ulbe) for discretization and wall nodes, Eq.(postcollision2_u) for
 * interpolation (interface) nodes, one forward-Euler sub-step of dt_u with all
 * right-hand sides at the old level (Jacobi: fout is a separate buffer).
 *
 * Eq.(postcollision2_u): the star quantities are the structured-derived ones
 * (f^eq,s and (1 - 1/(2 tau_s)) f^neq,s, passed in star_eq / star_neq) when
 * the neighbour is an interpolation node, and the grid's own f^eq, f^neq
 * otherwise; the leading term is the star value of the node itself.
 *
 * Wall nodes (reading; the paper states the rule for the refill only, Sec.
 * Refill procedure): after the Eq.(ulbe) update over the control volume closed
 * along the wall, the velocity is set to the wall velocity while the density
 * and the non-equilibrium part are kept: f <- f^eq(rho, u_w) + (f - f^eq(rho, u)). */
static void fv_substep_r(const or_mesh *m, const real *f, const real *star_eq,
                         const real *star_neq, real *fout, real tau_u,
                         double dt_u, const real *uwx, const real *uwy) {
  const int N = m->nnode;
  real *feq = malloc((size_t)9 * N * sizeof(real));
  /* per-node loops (same results on any number of threads) */
#pragma omp parallel for schedule(static) num_threads(or_threads) if (or_threads > 1)
  for (int p = 0; p < N; ++p) {
    real fp[9], e[9], rho, ux, uy;
    for (int i = 0; i < 9; ++i) fp[i] = f[(size_t)i * N + p];
    moments(fp, &rho, &ux, &uy);
    feq_r(rho, ux, uy, e);
    for (int i = 0; i < 9; ++i) feq[(size_t)i * N + p] = e[i];
  }
#pragma omp parallel for schedule(static) num_threads(or_threads) if (or_threads > 1)
  for (int p = 0; p < N; ++p) {
    const int iface = (m->type[p] == OR_NODE_INTERFACE);
    real out[9];
    for (int i = 0; i < 9; ++i) {
      real sum_s = 0.0, sum_c = 0.0, self;
      if (iface) self = star_eq[(size_t)i * N + p] + star_neq[(size_t)i * N + p];
      else self = f[(size_t)i * N + p];
      for (int k = 0; k < m->nk[p]; ++k) {
        const int q = m->nbr[p * KCAP + k];
        real fq, nq;
        if (iface && m->type[q] == OR_NODE_INTERFACE) {
          fq = star_eq[(size_t)i * N + q] + star_neq[(size_t)i * N + q];
          nq = star_neq[(size_t)i * N + q];
        } else {
          fq = f[(size_t)i * N + q];
          nq = f[(size_t)i * N + q] - feq[(size_t)i * N + q];
        }
        sum_s += m->S[((size_t)p * 9 + i) * KCAP + k] * fq;
        sum_c += m->C[p * KCAP + k] * nq;
      }
      out[i] = self + dt_u * sum_s - (dt_u / tau_u) * sum_c;
    }
    if (m->type[p] == OR_NODE_WALL) {
      real rho, ux, uy, e[9], ew[9];
      moments(out, &rho, &ux, &uy);
      feq_r(rho, ux, uy, e);
      feq_r(rho, uwx[p], uwy[p], ew);
      for (int i = 0; i < 9; ++i) out[i] = ew[i] + (out[i] - e[i]);
    }
    for (int i = 0; i < 9; ++i) fout[(size_t)i * N + p] = out[i];
  }
  free(feq);
}

#ifndef OR_COMPLEX_STEP
void or_fv_substep(const or_mesh *m, const double *f, const double *star_eq,
                   const double *star_neq, double *fout, double tau_u,
                   double dt_u, const double *uwx, const double *uwy) {
  fv_substep_r(m, f, star_eq, star_neq, fout, tau_u, dt_u, uwx, uwy);
}
#endif

/* Force on the body per unit depth (reading: the paper computes it on the
 * grid nodes lying on the body surface but gives no formula). Traction
 * t = -p' n + sigma' n with p' = c_s^2 (rho - 1) and the viscous stress of
 * the finite-volume populations sigma'_ab = -sum_i c_ia c_ib f_i^neq; the
 * grid's f^neq already carries the structured factor (1 - 1/(2 tau_s)) by
 * Eq.(continuity_stresses). n points out of the body; each wall edge is
 * integrated with the trapezoid rule. */
static void mesh_force_r(const or_mesh *m, const real *f, real F[2]) {
  const int N = m->nnode;
  F[0] = 0.0;
  F[1] = 0.0;
  for (int e = 0; e < m->nwe; ++e) {
    const double nx = m->wn[2 * e], ny = m->wn[2 * e + 1];
    real tx = 0.0, ty = 0.0;
    for (int s = 0; s < 2; ++s) {
      const int p = m->we[2 * e + s];
      real fp[9], eq[9], rho, ux, uy;
      for (int i = 0; i < 9; ++i) fp[i] = f[(size_t)i * N + p];
      moments(fp, &rho, &ux, &uy);
      feq_r(rho, ux, uy, eq);
      real sxx = 0.0, sxy = 0.0, syy = 0.0;
      for (int i = 0; i < 9; ++i) {
        const real fn = fp[i] - eq[i];
        sxx -= CX[i] * CX[i] * fn;
        sxy -= CX[i] * CY[i] * fn;
        syy -= CY[i] * CY[i] * fn;
      }
      const real pp = CS2 * (rho - 1.0);
      tx += -pp * nx + sxx * nx + sxy * ny;
      ty += -pp * ny + sxy * nx + syy * ny;
    }
    F[0] += 0.5 * m->wl[e] * tx;
    F[1] += 0.5 * m->wl[e] * ty;
  }
}

#ifndef OR_COMPLEX_STEP
void or_mesh_force(const or_mesh *m, const double *f, double F[2]) { mesh_force_r(m, f, F); }
#endif

/* ------------------------------------------------------------------ */
/* The hybrid method                                                   */
/* ------------------------------------------------------------------ */
struct or_sim {
  int nx, ny, nux, nuy, bc, n;
  double h, b, T, nu, dt_u, xc, yc, margin;
  real tau_s, tau_u, A, omega;  /* the differentiable parameters */
  double kc, beta;
  double body_b; /* width of the meshed-out lamina slot (0: no body) */
  int64_t k;
  real *fA, *fB;            /* lattice [9][ny][nx] */
  uint8_t *disc;            /* lattice discretization flags of this step */
  or_mesh *m;
  real *fu, *fu2;           /* grid populations [9][nnode] */
  real *star_eq, *star_neq;
  real *uwx, *uwy;
  real *hist;
  int64_t hist_cap, hist_n;
  int64_t nt1, nt2, nt3;
  double ex0, ex1, ey0, ey1; /* local extents of the grid's nodes */
  /* two-way coupled motion (or_set_motion): M y'' + C y' + K y = F_y */
  int fsi;
  double M, Ks, Cd, y_max;
  double y_cur, y_prev, v_cur;
  double *mhist; /* [hist_cap + 1][2]: (y, v) at t_k */
  int plant;             /* OR_FLAG_PLANT_* (tests only) */
  double u_bot, u_top;   /* tangential velocities of the lattice's y walls */
  /* wall band (or_create_wallband): a static grid on a tangentially
   * oscillating wall, periodic in x, in place of the lamina grid */
  int band;
  double band_U, band_omega;
  /* a given triangulation (or_create_mesh) and its prescribed deformation
   * (or_set_deformation): node p's local y is yref[p] + prof[p] beta_k */
  int unstructured;
  int deform;
  double dB, dphi;
  double *yref, *prof, *sx;
};

/* prescribed motion y(t) = A sin(omega t) (Sec. Problem statement), t = k */
static real motion_y(const or_sim *s, int64_t k) { return s->A * RSIN(s->omega * (double)k); }

/* Fictitious curve (reading: the paper draws it inside the grid boundary but
 * gives no construction): the axis-aligned rectangle of the grid's node
 * bounding box at offset y, inset by a margin of 2 lattice units. */
typedef struct { double x0, x1, y0, y1; } rect_t;

static rect_t rect_at(const or_sim *s, double y) {
  rect_t r;
  r.x0 = s->xc + s->ex0 + s->margin;
  r.x1 = s->xc + s->ex1 - s->margin;
  r.y0 = s->yc + y + s->ey0 + s->margin;
  r.y1 = s->yc + y + s->ey1 - s->margin;
  return r;
}

static int inside_rect(const rect_t *r, int x, int y) {
  return (double)x >= r->x0 && (double)x <= r->x1 && (double)y >= r->y0 && (double)y <= r->y1;
}

/* Node classes of the lattice (Sec. Refill procedure): nodes inside the
 * fictitious curve are unused, unless one of their eight lattice neighbours is
 * a discretization node, which makes them interpolation nodes. */
static int lattice_status(const rect_t *r, int x, int y) {
  if (!inside_rect(r, x, y)) return 0;
  for (int i = 1; i < 9; ++i)
    if (!inside_rect(r, x + CX[i], y + CY[i])) return 1;
  return 2;
}

int or_set_walls(or_sim *s, double u_bot, double u_top) {
  if (!s || s->bc != OR_BC_PERIODIC_X_WALLS_Y) return OR_E_ARG;
  s->u_bot = u_bot;
  s->u_top = u_top;
  return OR_OK;
}

int32_t or_lattice_status(const or_sim *s, int64_t k, int32_t x, int32_t y) {
  if (!s->m) return 0;
  rect_t r = rect_at(s, RE(motion_y(s, k)));
  return lattice_status(&r, x, y);
}

static void free_sim(or_sim *s) {
  if (!s) return;
  free(s->fA); free(s->fB); free(s->disc); or_mesh_free(s->m);
  free(s->fu); free(s->fu2); free(s->star_eq); free(s->star_neq);
  free(s->uwx); free(s->uwy); free(s->hist); free(s->mhist);
  free(s->yref); free(s->prof); free(s->sx);
  free(s);
}

void or_destroy(or_sim *s) { free_sim(s); }

/* X, Y: columns and rows of a graded grid (or_create_graded), or NULL;
 * M: a finished mesh of any triangulation (or_create_mesh), or NULL; the
 * case owns it from here on */
static int create_sim(const or_config *c, const double *X, const double *Y, or_mesh *M, or_sim **out) {
  if (!c || !out) {
    or_mesh_free(M);
    return OR_E_ARG;
  }
  *out = NULL;
  if (c->nx < 3 || c->ny < 3 || !(c->tau > 0.5) || c->max_steps < 0 ||
      (c->bc != OR_BC_PERIODIC_X_WALLS_Y && c->bc != OR_BC_PERIODIC && c->bc != OR_BC_PAPER &&
       c->bc != OR_BC_RING)) {
    or_mesh_free(M);
    return OR_E_ARG;
  }
  const int has_mesh = (c->nux > 0 || c->nuy > 0) || M;
  const int body = has_mesh && c->b > 0.0 && !(c->flags & OR_FLAG_NO_BODY);
  or_sim *s = xcalloc(1, sizeof(or_sim));
  if (!s) {
    or_mesh_free(M);
    return OR_E_NOMEM;
  }
  s->m = M;
  s->plant = c->flags & (OR_FLAG_PLANT_S_FACTOR | OR_FLAG_PLANT_NO_KNEQ | OR_FLAG_PLANT_SWAP_BILIN_Y |
                         OR_FLAG_PLANT_SWAP_BILIN_X | OR_FLAG_PLANT_BARY);
  s->nx = c->nx;
  s->ny = c->ny;
  s->nux = c->nux;
  s->nuy = c->nuy;
  s->bc = c->bc;
  s->h = (c->h_u > 0.0) ? c->h_u : 1.0;
  s->b = c->b;
  s->body_b = body ? c->b : 0.0;
  s->kc = c->kc;
  s->beta = c->beta;
  s->tau_s = c->tau;
  /* viscosity matching (Sec. 3): nu = c_s^2 (tau_s - 1/2) on the lattice and
   * nu = c_s^2 tau_u on the grid, hence tau_u = tau_s - 1/2 */
  s->nu = (c->tau - 0.5) / 3.0;
  s->tau_u = c->tau - 0.5;
  /* Sec. Problem statement: KC = 2 pi eps = 2 pi A / L, beta = omega L^2 / (2 pi nu) */
  if (has_mesh && c->b > 0.0) {
    s->A = c->kc * c->b / (2.0 * M_PI);
    s->omega = 2.0 * M_PI * s->nu * c->beta / (c->b * c->b);
  } else {
    s->A = 0.0;
    s->omega = 0.0;
  }
  /* sub-steps: Delta t_s = n Delta t_u; automatic n keeps Delta t_u <= tau_u,
   * half the explicit stability bound Delta t < 2 tau (Sec. Numerical
   * performance) */
  if (c->n_sub > 0) s->n = c->n_sub;
  else {
    int n = (int)ceil(1.0 / RE(s->tau_u) - 1e-9);
    s->n = n < 2 ? 2 : n;
  }
  s->dt_u = 1.0 / (double)s->n;
  s->xc = (double)(c->nx / 2);
  s->yc = 0.5 * (double)(c->ny - 1);
  s->margin = 2.0;
  s->hist_cap = c->max_steps;
  const size_t L = (size_t)9 * c->nx * c->ny;
  s->fA = malloc(L * sizeof(real));
  s->fB = malloc(L * sizeof(real));
  s->disc = malloc((size_t)c->nx * c->ny);
  s->hist = xcalloc((size_t)2 * (c->max_steps > 0 ? c->max_steps : 1), sizeof(real));
  if (!s->fA || !s->fB || !s->disc || !s->hist) {
    free_sim(s);
    return OR_E_NOMEM;
  }
  /* initial state (reading): fluid at rest with unit density everywhere */
  for (int i = 0; i < 9; ++i)
    for (size_t p = 0; p < (size_t)c->nx * c->ny; ++p) {
      s->fA[(size_t)i * c->nx * c->ny + p] = WT[i];
      s->fB[(size_t)i * c->nx * c->ny + p] = WT[i];
    }
  if (has_mesh) {
    if (X && (c->nux < 4 || c->nuy < 4 || (c->nuy % 2) != 0)) { free_sim(s); return OR_E_ARG; }
    if (X)
      for (int j = 0; j < c->nuy; ++j)
        if (Y[j] != -Y[c->nuy - 1 - j]) { free_sim(s); return OR_E_ARG; } /* rows symmetric about the lamina */
    /* thickness of the lamina slot (a given triangulation: as configured) */
    const double Tg = M ? c->thickness : X ? Y[c->nuy / 2] - Y[c->nuy / 2 - 1] : s->h;
    if (body && fabs(c->thickness - Tg) > 1e-12 * Tg) { free_sim(s); return OR_E_ARG; }
    if (c->n_sub < 0) { free_sim(s); return OR_E_ARG; }
    /* explicit stability of the grid scheme, Delta t_u < 2 tau_u */
    if (!(s->dt_u < 2.0 * RE(s->tau_u))) { free_sim(s); return OR_E_ARG; }
    if (M) {
      /* the grid's outer boundary is the bounding box of its nodes */
      s->ex0 = s->ey0 = 1e300;
      s->ex1 = s->ey1 = -1e300;
      for (int p = 0; p < M->nnode; ++p) {
        s->ex0 = fmin(s->ex0, M->x[p]);
        s->ex1 = fmax(s->ex1, M->x[p]);
        s->ey0 = fmin(s->ey0, M->y[p]);
        s->ey1 = fmax(s->ey1, M->y[p]);
      }
      if (!(s->ey1 > 0.0 && s->ey0 < 0.0 && fabs(s->ey0 + s->ey1) <= 1e-12 * s->ey1)) {
        free_sim(s); /* rows symmetric about the lamina, as the other grids */
        return OR_E_ARG;
      }
    } else if (X) {
      s->m = or_mesh_lamina_coords(c->nux, c->nuy, X, Y, s->body_b);
      s->ex0 = X[0];
      s->ex1 = X[c->nux - 1];
      s->ey0 = Y[0];
      s->ey1 = Y[c->nuy - 1];
    } else {
      s->m = or_mesh_lamina(c->nux, c->nuy, s->h, s->body_b);
      s->ex0 = (double)(0 - c->nux / 2) * s->h;
      s->ex1 = (double)(c->nux - 1 - c->nux / 2) * s->h;
      s->ey0 = (0.0 - 0.5 * (double)(c->nuy - 1)) * s->h;
      s->ey1 = ((double)(c->nuy - 1) - 0.5 * (double)(c->nuy - 1)) * s->h;
    }
    if (!s->m) { free_sim(s); return OR_E_ARG; }
    s->T = s->m->T;
    /* geometric requirements: the grid and the lattice donors of its outer
     * nodes stay inside the lattice; the fictitious rectangle holds the body
     * with a one-unit gap; a node moves less than one lattice unit per step */
    const double hx = -s->ex0, hxr = s->ex1;
    const double hy = s->ey1;
    if (s->xc - hx < 1.0 || s->xc + hxr > (double)c->nx - 2.0) { free_sim(s); return OR_E_ARG; }
    if (c->bc != OR_BC_PERIODIC &&
        (s->yc - hy - fabs(RE(s->A)) < 1.0 || s->yc + hy + fabs(RE(s->A)) > (double)c->ny - 2.0)) {
      free_sim(s);
      return OR_E_ARG;
    }
    if (body && (0.5 * c->b + 1.0 > hx - s->margin - 1.0 || 0.5 * c->b + 1.0 > hxr - s->margin - 1.0 ||
                       0.5 * Tg + 1.0 > hy - s->margin - 1.0)) {
      free_sim(s);
      return OR_E_ARG;
    }
    if (!(fabs(RE(s->A * s->omega)) < 1.0)) { free_sim(s); return OR_E_ARG; }
    const int N = s->m->nnode;
    s->fu = malloc((size_t)9 * N * sizeof(real));
    s->fu2 = malloc((size_t)9 * N * sizeof(real));
    s->star_eq = xcalloc((size_t)9 * N, sizeof(real));
    s->star_neq = xcalloc((size_t)9 * N, sizeof(real));
    s->uwx = xcalloc(N, sizeof(real));
    s->uwy = xcalloc(N, sizeof(real));
    if (!s->fu || !s->fu2 || !s->star_eq || !s->star_neq || !s->uwx || !s->uwy) {
      free_sim(s);
      return OR_E_NOMEM;
    }
    for (int i = 0; i < 9; ++i)
      for (int p = 0; p < N; ++p) s->fu[(size_t)i * N + p] = WT[i];
  }
  *out = s;
  return OR_OK;
}

int or_create(const or_config *c, or_sim **out) { return create_sim(c, NULL, NULL, NULL, out); }

/* A case on a given triangulation (see the header): the mesh is copied,
 * its matrices and buckets built by the same routines as the lamina grid's,
 * the lamina geometry (b, thickness) taken from the configuration. */
int or_create_mesh(const or_config *c, int32_t nnode, const double *xy, const int32_t *type, int32_t ntri,
                   const int32_t *tri, or_sim **out) {
  if (!c || !out || !xy || !type || !tri || nnode < 3 || ntri < 1) return OR_E_ARG;
  *out = NULL;
  or_mesh *m = mesh_alloc(nnode, ntri);
  if (!m) return OR_E_NOMEM;
  int nwall = 0, nface = 0;
  for (int p = 0; p < nnode; ++p) {
    if (type[p] != OR_NODE_INTERIOR && type[p] != OR_NODE_INTERFACE && type[p] != OR_NODE_WALL) {
      or_mesh_free(m);
      return OR_E_ARG;
    }
    m->x[p] = xy[2 * p];
    m->y[p] = xy[2 * p + 1];
    m->type[p] = type[p];
    nwall += type[p] == OR_NODE_WALL;
    nface += type[p] == OR_NODE_INTERFACE;
  }
  for (int t = 0; t < ntri; ++t)
    for (int a = 0; a < 3; ++a) {
      const int id = tri[3 * t + a];
      if (id < 0 || id >= nnode) {
        or_mesh_free(m);
        return OR_E_ARG;
      }
      m->tri[3 * t + a] = id;
      m->txy[6 * t + 2 * a] = m->x[id];
      m->txy[6 * t + 2 * a + 1] = m->y[id];
    }
  m->ntri = ntri;
  const int body = c->b > 0.0 && !(c->flags & OR_FLAG_NO_BODY);
  if (nface == 0 || (body && nwall == 0) || (!body && nwall > 0)) {
    or_mesh_free(m);
    return OR_E_ARG;
  }
  m->b = body ? c->b : 0.0;
  m->T = body ? c->thickness : 0.0;
  m = mesh_finish(m); /* frees the mesh on failure (a triangle not counter-clockwise, ...) */
  if (!m) return OR_E_ARG;
  const int rc = create_sim(c, NULL, NULL, m, out);
  if (rc == OR_OK) (*out)->unstructured = 1;
  return rc;
}

/* A static grid band on a tangentially oscillating wall (see the header):
 * the lattice of create_sim without a lamina, then the band grid, its
 * arrays and the fictitious line y = y_wall + nband - 1 - margin. */
int or_create_wallband(const or_config *c, int32_t nband, double x_off, double y_wall, double U,
                       double omega, or_sim **out) {
  if (!c || !out) return OR_E_ARG;
  *out = NULL;
  if (c->bc != OR_BC_PERIODIC_X_WALLS_Y || nband < 4 || !(x_off >= 0.0 && x_off < 1.0) ||
      !(y_wall >= 0.0) || !(y_wall + nband + 2.0 < c->ny - 2.0) || c->n_sub < 0)
    return OR_E_ARG;
  or_config lc = *c;
  lc.nux = 0;
  lc.nuy = 0;
  lc.b = 0.0;
  or_sim *s = NULL;
  int rc = create_sim(&lc, NULL, NULL, NULL, &s);
  if (rc != OR_OK) return rc;
  if (!(s->dt_u < 2.0 * RE(s->tau_u))) { free_sim(s); return OR_E_ARG; }
  s->m = mesh_strip(c->nx, nband, 1.0, OR_NODE_INTERFACE);
  if (!s->m) { free_sim(s); return OR_E_ARG; }
  s->band = 1;
  s->band_U = U;
  s->band_omega = omega;
  s->nux = c->nx;
  s->nuy = nband;
  s->xc = x_off;
  s->yc = y_wall;
  s->ex0 = -1e300;
  s->ex1 = 1e300;
  s->ey0 = -1e300;
  s->ey1 = (double)(nband - 1);
  const int N = s->m->nnode;
  s->fu = malloc((size_t)9 * N * sizeof(real));
  s->fu2 = malloc((size_t)9 * N * sizeof(real));
  s->star_eq = xcalloc((size_t)9 * N, sizeof(real));
  s->star_neq = xcalloc((size_t)9 * N, sizeof(real));
  s->uwx = xcalloc(N, sizeof(real));
  s->uwy = xcalloc(N, sizeof(real));
  if (!s->fu || !s->fu2 || !s->star_eq || !s->star_neq || !s->uwx || !s->uwy) {
    free_sim(s);
    return OR_E_NOMEM;
  }
  for (int i = 0; i < 9; ++i)
    for (int p = 0; p < N; ++p) s->fu[(size_t)i * N + p] = WT[i];
  *out = s;
  return OR_OK;
}


/* threads of the per-node loops: 1 unless asked (1 without OpenMP); n <= 0
 * leaves the setting alone; returns the number in effect */
int or_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) or_threads = n;
  return or_threads;
#else
  (void)n;
  return 1;
#endif
}

/* A case whose grid has graded spacing: columns at local x = X[nux], rows at
 * y = Y[nuy] (or_mesh_lamina_coords; rows symmetric about the lamina, whose
 * thickness Y[nuy/2] - Y[nuy/2-1] must equal cfg->thickness; h_u unused). */
int or_create_graded(const or_config *c, const double *X, const double *Y, or_sim **out) {
  if (!X || !Y) return OR_E_ARG;
  return create_sim(c, X, Y, NULL, out);
}

/* lattice populations arriving at node (x,y) at t_{k+1}: pulled from the
 * post-collision buffer of t_k (the pre-collision f of Eq.(LBE)'s left side) */
static void lattice_pre(const or_sim *s, int x, int y, real f[9]) {
  pull_node(s->fA, s->nx, s->ny, s->bc, wrap(x, s->nx), s->bc == OR_BC_PERIODIC ? wrap(y, s->ny) : y,
            s->u_bot, s->u_top, f);
}

/* Bilinear Lagrange interpolation over the four lattice nodes of the cell
 * enclosing (X,Y) (Sec. Refill procedure, type 1): density, velocity and the
 * non-equilibrium part f^neq,s = f - f^eq(rho, u) of the pre-collision
 * populations at t_{k+1}. */
static void lattice_bilinear(const or_sim *s, double X, real Y, real *rho,
                             real *ux, real *uy, real fneq[9]) {
  const double fx = floor(X), fy = floor(RE(Y));
  const int x0 = (int)fx, y0 = (int)fy;
  real a = X - fx, bb = Y - fy;
  if (s->plant & OR_FLAG_PLANT_SWAP_BILIN_X) a = 1.0 - a;
  if (s->plant & OR_FLAG_PLANT_SWAP_BILIN_Y) bb = 1.0 - bb;
  const real wgt[4] = {(1.0 - a) * (1.0 - bb), a * (1.0 - bb), (1.0 - a) * bb, a * bb};
  const int dx[4] = {0, 1, 0, 1}, dy[4] = {0, 0, 1, 1};
  *rho = 0.0;
  *ux = 0.0;
  *uy = 0.0;
  for (int i = 0; i < 9; ++i) fneq[i] = 0.0;
  for (int d = 0; d < 4; ++d) {
    real f[9], e[9], r, vx, vy;
    lattice_pre(s, x0 + dx[d], y0 + dy[d], f);
    moments(f, &r, &vx, &vy);
    feq_r(r, vx, vy, e);
    *rho += wgt[d] * r;
    *ux += wgt[d] * vx;
    *uy += wgt[d] * vy;
    for (int i = 0; i < 9; ++i) fneq[i] += wgt[d] * (f[i] - e[i]);
  }
}

/* planted mistake (tests only): the barycentric weights in a rotated vertex
 * order */
static void plant_rotate(const or_sim *s, real lam[3]) {
  if (!(s->plant & OR_FLAG_PLANT_BARY)) return;
  const real l0 = lam[0];
  lam[0] = lam[1];
  lam[1] = lam[2];
  lam[2] = l0;
}

/* Barycentric interpolation of the grid at lattice position (X, Y) with the
 * grid at offset yk: density, velocity and f^neq,u = f^u - f^eq(rho^u, u^u)
 * over the enclosing triangle (Sec. Refill procedure: barycentric on the
 * grid; reading: the moments and f^neq are interpolated, f^eq is rebuilt
 * from the interpolated moments). A band grid is periodic in x. */
static int grid_interp(const or_sim *s, double X, real Y, real yk, real *rho, real *ux, real *uy,
                       real fneq[9]) {
  const or_mesh *m = s->m;
  const int N = m->nnode;
  double lam0[3];
  double px = X - s->xc;
  if (s->band) px -= (double)s->nx * floor(px / (double)s->nx);
  const real py = Y - (s->yc + yk);
  const int t = or_mesh_locate(m, px, RE(py), lam0);
  if (t < 0) return OR_E_STATE;
  real lam[3];
  bary_r(&m->txy[6 * t], px, py, lam);
  plant_rotate(s, lam);
  *rho = 0.0;
  *ux = 0.0;
  *uy = 0.0;
  for (int i = 0; i < 9; ++i) fneq[i] = 0.0;
  for (int a = 0; a < 3; ++a) {
    const int p = m->tri[3 * t + a];
    real f[9], e[9], r, vx, vy;
    for (int i = 0; i < 9; ++i) f[i] = s->fu[(size_t)i * N + p];
    moments(f, &r, &vx, &vy);
    feq_r(r, vx, vy, e);
    *rho += lam[a] * r;
    *ux += lam[a] * vx;
    *uy += lam[a] * vy;
    for (int i = 0; i < 9; ++i) fneq[i] += lam[a] * (f[i] - e[i]);
  }
  return OR_OK;
}

/* Eq.(postcollision2_s) at lattice node (x,y) from the grid at offset y_k:
 * the interpolated moments and f^neq,u of grid_interp, written as the
 * post-collision populations f^eq + 2 (tau_s - 1)/(2 tau_s - 1) f^neq,u. */
static int lattice_from_grid(or_sim *s, int x, int y, real yk) {
  real rho, ux, uy, fneq[9];
  if (grid_interp(s, (double)x, (double)y, yk, &rho, &ux, &uy, fneq) != OR_OK) return OR_E_STATE;
  real e[9];
  feq_r(rho, ux, uy, e);
  const real g = (s->plant & OR_FLAG_PLANT_S_FACTOR) ? 1.0 - 1.0 / s->tau_s
                                                     : 2.0 * (s->tau_s - 1.0) / (2.0 * s->tau_s - 1.0);
  for (int i = 0; i < 9; ++i) s->fA[lidx(s->nx, s->ny, i, x, y)] = e[i] + g * fneq[i];
  return OR_OK;
}

#ifndef OR_COMPLEX_STEP
int or_probe_bilinear(const or_sim *s, double X, double Y, double out[12]) {
  if (!s || !out) return OR_E_ARG;
  real rho, ux, uy, fneq[9];
  lattice_bilinear(s, X, Y, &rho, &ux, &uy, fneq);
  out[0] = rho;
  out[1] = ux;
  out[2] = uy;
  for (int i = 0; i < 9; ++i) out[3 + i] = fneq[i];
  return OR_OK;
}

int or_probe_grid(const or_sim *s, double X, double Y, double out[12]) {
  if (!s || !out || !s->m) return OR_E_ARG;
  real rho, ux, uy, fneq[9];
  const real yk = s->fsi ? s->y_cur : motion_y(s, s->k);
  if (grid_interp(s, X, Y, yk, &rho, &ux, &uy, fneq) != OR_OK) return OR_E_STATE;
  out[0] = rho;
  out[1] = ux;
  out[2] = uy;
  for (int i = 0; i < 9; ++i) out[3 + i] = fneq[i];
  return OR_OK;
}
#endif

/* Prescribed deformation (the extension to deformable bodies that Sec.
 * Conclusions names; reading of this build): the lamina's centreline moves
 * as Y(x, t) = A sin(omega t) + B sin(omega t + phi) s(x), with s = (2x/b)^2
 * on the lamina, so it bends symmetrically about its centre. The grid
 * follows: node p, at local (x, y) in the reference triangulation, sits at
 * y + s(x) w(y) beta(t), beta = B sin(omega t + phi), in the frame that
 * moves with A sin(omega t); s falls linearly from 1 at |x| = b/2 to 0 at
 * the grid's side, w is 1 for |y| <= T/2 and falls linearly to 0 at its top
 * and bottom, so the outer boundary moves rigidly and the lamina keeps its
 * vertical thickness T. The grid is static during the sub-steps of a step
 * (at beta_k); its matrices, wall edges and triangles are those of that
 * configuration. Not differentiated (the complex-step build deforms with
 * the real part of omega). */
static double deform_s(const or_sim *s, double x) {
  const double hb = 0.5 * s->b;
  if (fabs(x) <= hb) return (x / hb) * (x / hb);
  const double xr = x < 0.0 ? -s->ex0 : s->ex1;
  const double r = 1.0 - (fabs(x) - hb) / (xr - hb);
  return r > 0.0 ? r : 0.0;
}

static double deform_w(const or_sim *s, double y) {
  const double ht = 0.5 * s->T;
  if (fabs(y) <= ht) return 1.0;
  const double r = 1.0 - (fabs(y) - ht) / (s->ey1 - ht);
  return r > 0.0 ? r : 0.0;
}

static double deform_beta(const or_sim *s, int64_t k) {
  return s->dB * sin(RE(s->omega) * (double)k + s->dphi);
}

/* the grid in the configuration beta: node positions, triangles, matrices
 * and wall edges */
static int set_geometry(or_sim *s, double beta) {
  or_mesh *m = s->m;
  for (int p = 0; p < m->nnode; ++p) m->y[p] = s->yref[p] + s->prof[p] * beta;
  for (int t = 0; t < m->ntri; ++t)
    for (int a = 0; a < 3; ++a) m->txy[6 * t + 2 * a + 1] = m->y[m->tri[3 * t + a]];
  free(m->nk); free(m->nbr); free(m->S); free(m->C); free(m->V);
  free(m->we); free(m->wn); free(m->wl);
  m->nk = NULL; m->nbr = NULL; m->S = NULL; m->C = NULL; m->V = NULL;
  m->we = NULL; m->wn = NULL; m->wl = NULL;
  return assemble(m);
}

int or_set_deformation(or_sim *s, double B, double phi) {
  if (!s || !s->unstructured || s->k != 0 || s->fsi || !(s->b > 0.0) || !(fabs(B) < 1.0)) return OR_E_ARG;
  const double ht = 0.5 * s->T;
  if (!(fabs(B) < s->ey1 - ht)) return OR_E_ARG;
  /* the deflected lamina stays inside the fictitious rectangle, and no node
   * moves a lattice unit per step */
  if (!(ht + fabs(B) + 1.0 <= s->ey1 - s->margin - 1.0)) return OR_E_ARG;
  if (!(fabs(RE(s->A * s->omega)) + fabs(B * RE(s->omega)) < 1.0)) return OR_E_ARG;
  or_mesh *m = s->m;
  const int N = m->nnode;
  s->yref = malloc((size_t)N * sizeof(double));
  s->prof = malloc((size_t)N * sizeof(double));
  s->sx = malloc((size_t)N * sizeof(double));
  if (!s->yref || !s->prof || !s->sx) return OR_E_NOMEM;
  for (int p = 0; p < N; ++p) {
    s->yref[p] = m->y[p];
    s->sx[p] = deform_s(s, m->x[p]);
    s->prof[p] = s->sx[p] * deform_w(s, m->y[p]);
  }
  /* a triangle's area is linear in beta: positive at both extremes, positive
   * throughout */
  for (int e = -1; e <= 1; e += 2)
    for (int t = 0; t < m->ntri; ++t) {
      double y[3];
      const double *q = &m->txy[6 * t];
      for (int a = 0; a < 3; ++a) y[a] = s->yref[m->tri[3 * t + a]] + s->prof[m->tri[3 * t + a]] * e * B;
      if (!((q[2] - q[0]) * (y[2] - y[0]) - (q[4] - q[0]) * (y[1] - y[0]) > 0.0)) return OR_E_ARG;
    }
  s->dB = B;
  s->dphi = phi;
  s->deform = 1;
  return set_geometry(s, deform_beta(s, 0));
}

/* Refill after the move from y_k to y_k1 (Sec. Refill procedure). */
static void refill(or_sim *s, real yk, real yk1) {
  const or_mesh *m = s->m;
  const int N = m->nnode;
  /* Eq.(continuity_stresses) */
  const real kneq = (s->plant & OR_FLAG_PLANT_NO_KNEQ) ? 1.0 : 1.0 - 1.0 / (2.0 * s->tau_s);
  for (int p = 0; p < N; ++p) {
    real out[9];
    if (m->type[p] == OR_NODE_WALL) {
      /* wall nodes keep density and populations; their velocity is imposed
       * during the sub-steps */
      for (int i = 0; i < 9; ++i) out[i] = s->fu[(size_t)i * N + p];
    } else {
      const double X = s->xc + m->x[p];
      /* deformation: the node's own new local y */
      const double ynew = s->deform ? s->yref[p] + s->prof[p] * deform_beta(s, s->k + 1) : m->y[p];
      const real Ynew = (s->yc + yk1) + ynew;
      const real py = Ynew - (s->yc + yk);
      /* the old lamina's centreline under the node */
      const double yb = s->deform ? deform_beta(s, s->k) * deform_s(s, X - s->xc) : 0.0;
      double lam0[3];
      real lam[3];
      const int t = or_mesh_locate(m, X - s->xc, RE(py), lam0);
      if (t >= 0) {
        bary_r(&m->txy[6 * t], X - s->xc, py, lam);
        plant_rotate(s, lam);
      }
      if (t >= 0) {
        /* type 3: barycentric interpolation in the old triangle */
        for (int i = 0; i < 9; ++i) {
          out[i] = 0.0;
          for (int a = 0; a < 3; ++a) out[i] += lam[a] * s->fu[(size_t)i * N + m->tri[3 * t + a]];
        }
        s->nt3++;
      } else if (s->body_b > 0.0 && fabs(X - s->xc) < 0.5 * s->body_b && fabs(RE(py) - yb) < 0.5 * s->T) {
        /* type 2: inside the old body, keep the previous values */
        for (int i = 0; i < 9; ++i) out[i] = s->fu[(size_t)i * N + p];
        s->nt2++;
      } else {
        /* type 1: outside the old grid, from the lattice */
        real rho, ux, uy, fneq[9], e[9];
        lattice_bilinear(s, X, Ynew, &rho, &ux, &uy, fneq);
        feq_r(rho, ux, uy, e);
        for (int i = 0; i < 9; ++i) out[i] = e[i] + kneq * fneq[i];
        s->nt1++;
      }
    }
    for (int i = 0; i < 9; ++i) s->fu2[(size_t)i * N + p] = out[i];
  }
  real *tmp = s->fu;
  s->fu = s->fu2;
  s->fu2 = tmp;
}

int or_step(or_sim *s, int64_t nsteps) {
  if (!s || nsteps < 0) return OR_E_ARG;
  if (s->m && s->hist_n + nsteps > s->hist_cap) return OR_E_ARG;
  const int nx = s->nx, ny = s->ny;
  for (int64_t it = 0; it < nsteps; ++it) {
    const int64_t k = s->k;
    if (!s->m) {
      lattice_step_r(s->fA, s->fB, nx, ny, s->bc, s->tau_s, s->u_bot, s->u_top, NULL);
    } else {
      const or_mesh *m = s->m;
      const int N = m->nnode;
      /* lamina offset at t_k and t_{k-1}: prescribed, or the coupled state */
      const real yk = s->fsi ? s->y_cur : motion_y(s, k);
      const real yprev = s->fsi ? s->y_prev : ((k > 0) ? motion_y(s, k - 1) : yk);
      real yk1 = s->fsi ? 0.0 : motion_y(s, k + 1);
      const rect_t R = rect_at(s, RE(yk)), Rp = rect_at(s, RE(yprev));
      if (s->deform && set_geometry(s, deform_beta(s, k)) != OR_OK) return OR_E_STATE;
      /* 1. lattice interpolation nodes, plus nodes the moving fictitious line
       *    has just uncovered (Sec. Refill procedure, last paragraphs), get
       *    Eq.(postcollision2_s) from the grid at y_k */
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const int st = lattice_status(&R, x, y), sp = lattice_status(&Rp, x, y);
          s->disc[(size_t)y * nx + x] = (st == 0);
          if (st == 1 || (st == 0 && sp != 0))
            if (lattice_from_grid(s, x, y, yk) != OR_OK) return OR_E_STATE;
        }
      /* 2. Eq.(LBE) on the discretization nodes */
      lattice_step_r(s->fA, s->fB, nx, ny, s->bc, s->tau_s, s->u_bot, s->u_top, s->disc);
      /* 3. structured-derived values at the grid's outer nodes, from the
       *    lattice at t_{k+1} (pre-collision), held over the n sub-steps */
      const real kneq = (s->plant & OR_FLAG_PLANT_NO_KNEQ) ? 1.0 : 1.0 - 1.0 / (2.0 * s->tau_s);
      for (int p = 0; p < N; ++p) {
        if (m->type[p] != OR_NODE_INTERFACE) continue;
        real rho, ux, uy, fneq[9], e[9];
        lattice_bilinear(s, s->xc + m->x[p], (s->yc + yk) + m->y[p], &rho, &ux, &uy, fneq);
        feq_r(rho, ux, uy, e);
        for (int i = 0; i < 9; ++i) {
          s->star_eq[(size_t)i * N + p] = e[i];
          s->star_neq[(size_t)i * N + p] = kneq * fneq[i];
        }
      }
      /* 4. n sub-steps of the grid scheme, Delta t_s = n Delta t_u; the wall
       *    moves with the lamina, u_w = A omega cos(omega t) at the end of
       *    each sub-step */
      for (int sub = 0; sub < s->n; ++sub) {
        const double t = (double)k + (double)(sub + 1) / (double)s->n;
        /* coupled motion: the lamina keeps the velocity of t_k over the step */
        const real uw = s->fsi ? s->v_cur : s->A * s->omega * RCOS(s->omega * t);
        for (int p = 0; p < N; ++p) {
          s->uwx[p] = 0.0;
          s->uwy[p] = uw;
        }
        if (s->deform) /* the wall's own bending velocity */
          for (int p = 0; p < N; ++p)
            s->uwy[p] += s->dB * RE(s->omega) * cos(RE(s->omega) * t + s->dphi) * s->sx[p];
        if (s->band) /* the band's wall moves tangentially */
          for (int p = 0; p < N; ++p) {
            s->uwx[p] = s->band_U * cos(s->band_omega * t);
            s->uwy[p] = 0.0;
          }
        fv_substep_r(m, s->fu, s->star_eq, s->star_neq, s->fu2, s->tau_u, s->dt_u, s->uwx, s->uwy);
        real *tmp = s->fu;
        s->fu = s->fu2;
        s->fu2 = tmp;
      }
      /* 5. force on the lamina at t_{k+1} */
      real F[2];
      mesh_force_r(m, s->fu, F);
      s->hist[2 * s->hist_n] = F[0];
      s->hist[2 * s->hist_n + 1] = F[1];
      s->hist_n++;
      if (!isfinite(RE(F[0])) || !isfinite(RE(F[1]))) return OR_E_UNSTABLE;
#ifndef OR_COMPLEX_STEP
      if (s->fsi) {
        /* the body's equation of motion, semi-implicit Euler with Delta t = 1:
         * the force at t_{k+1} and the state at t_k give v_{k+1}, then
         * y_{k+1} = y_k + v_{k+1} */
        const double acc = (F[1] - s->Ks * s->y_cur - s->Cd * s->v_cur) / s->M;
        const double v1 = s->v_cur + acc;
        const double y1 = s->y_cur + v1;
        if (!(fabs(y1) <= s->y_max) || !(fabs(v1) < 1.0)) return OR_E_UNSTABLE;
        yk1 = y1;
        s->y_prev = s->y_cur;
        s->y_cur = y1;
        s->v_cur = v1;
        s->mhist[2 * (s->hist_n - 1)] = y1; /* the entry of this step's force */
        s->mhist[2 * (s->hist_n - 1) + 1] = v1;
      }
#endif
      /* 6. move the grid to y_{k+1} and refill it (a wall band stays put) */
      if (!s->band) refill(s, yk, yk1);
    }
    real *tmp = s->fA;
    s->fA = s->fB;
    s->fB = tmp;
    s->k = k + 1;
  }
  /* unstable if any density is not finite and positive */
  const size_t L = (size_t)nx * ny;
  for (size_t p = 0; p < L; ++p) {
    double r = 0.0;
    for (int i = 0; i < 9; ++i) r += RE(s->fA[(size_t)i * L + p]);
    if (!(r > 0.0) || !isfinite(r)) return OR_E_UNSTABLE;
  }
  return OR_OK;
}

int or_info_get(const or_sim *s, or_info *o) {
  if (!s || !o) return OR_E_ARG;
  memset(o, 0, sizeof(*o));
  const double A = RE(s->A), omega = RE(s->omega);
  o->nu = s->nu;
  o->tau_u = RE(s->tau_u);
  o->dt_u = s->dt_u;
  o->A = A;
  o->omega = omega;
  o->period = (omega > 0.0) ? 2.0 * M_PI / omega : 0.0;
  o->u_max = A * omega;
  o->mach = o->u_max * sqrt(3.0);
  o->reynolds = (s->nu > 0.0) ? o->u_max * s->b / s->nu : 0.0;
  o->eps = (s->b > 0.0) ? A / s->b : 0.0;
  o->beta_limit_ok = (o->eps > 0.0) ? (s->beta < 2.6 * pow(o->eps, -1.6)) : 1;
  o->n_sub = s->n;
  o->step = s->k;
  o->y = s->fsi ? s->y_cur : RE(motion_y(s, s->k));
  o->n_type1 = s->nt1;
  o->n_type2 = s->nt2;
  o->n_type3 = s->nt3;
  if (s->m) {
    o->nnode = s->m->nnode;
    o->ntri = s->m->ntri;
    o->n_wall_edges = s->m->nwe;
    for (int p = 0; p < s->m->nnode; ++p) {
      o->n_interface += s->m->type[p] == OR_NODE_INTERFACE;
      o->n_wall += s->m->type[p] == OR_NODE_WALL;
    }
  }
  return OR_OK;
}

const or_mesh *or_sim_mesh(const or_sim *s) { return s->m; }

#ifndef OR_COMPLEX_STEP
int or_get_lattice(const or_sim *s, double *out) {
  memcpy(out, s->fA, (size_t)9 * s->nx * s->ny * sizeof(double));
  return OR_OK;
}
int or_set_lattice(or_sim *s, const double *in) {
  memcpy(s->fA, in, (size_t)9 * s->nx * s->ny * sizeof(double));
  return OR_OK;
}
int or_get_mesh(const or_sim *s, double *out) {
  if (!s->m) return OR_E_STATE;
  memcpy(out, s->fu, (size_t)9 * s->m->nnode * sizeof(double));
  return OR_OK;
}
int or_set_mesh(or_sim *s, const double *in) {
  if (!s->m) return OR_E_STATE;
  memcpy(s->fu, in, (size_t)9 * s->m->nnode * sizeof(double));
  return OR_OK;
}
/* Two-way coupled motion instead of the prescribed one (before the first
 * step; a grid with the lamina): the lamina, of mass M per unit depth on a
 * spring K and damper C, moves under the y-force of the fluid. The state
 * starts at (y0, v0); |y| may not exceed y_max, which the geometric checks
 * of or_create take in place of the amplitude A. */
int or_set_motion(or_sim *s, double M, double K, double C, double y0, double v0, double y_max) {
  if (!s || !s->m || !(s->body_b > 0.0) || s->k != 0) return OR_E_STATE;
  if (!(M > 0.0) || !(K >= 0.0) || !(C >= 0.0) || !(y_max > 0.0) || !(fabs(y0) <= y_max) || !(fabs(v0) < 1.0))
    return OR_E_ARG;
  if (s->bc != OR_BC_PERIODIC && (s->yc + s->ey0 - y_max < 1.0 || s->yc + s->ey1 + y_max > (double)s->ny - 2.0))
    return OR_E_ARG;
  double *mh = calloc((size_t)2 * (s->hist_cap + 1), sizeof(double));
  if (!mh) return OR_E_NOMEM;
  free(s->mhist);
  s->mhist = mh;
  s->fsi = 1;
  s->M = M;
  s->Ks = K;
  s->Cd = C;
  s->y_max = y_max;
  s->y_cur = s->y_prev = y0;
  s->v_cur = v0;
  return OR_OK;
}

/* (y, v) after each step: entry k at t = k+1; returns the count */
int64_t or_motion_history(const or_sim *s, double *out, int64_t cap) {
  if (!s->fsi) return 0;
  const int64_t n = s->hist_n < cap ? s->hist_n : cap;
  if (out) memcpy(out, s->mhist, (size_t)2 * n * sizeof(double));
  return s->hist_n;
}

int64_t or_history(const or_sim *s, double *out, int64_t cap) {
  const int64_t n = s->hist_n < cap ? s->hist_n : cap;
  if (out) memcpy(out, s->hist, (size_t)2 * n * sizeof(double));
  return s->hist_n;
}
#else
/* complex-step build: add i h to A, omega and tau_s (tau_u follows) */
int or_cs_perturb(or_sim *s, double hA, double homega, double htau) {
  s->A += I * hA;
  s->omega += I * homega;
  s->tau_s += I * htau;
  s->tau_u = s->tau_s - 0.5;
  return OR_OK;
}
static void split(const real *src, size_t n, double *re, double *im) {
  for (size_t i = 0; i < n; ++i) {
    if (re) re[i] = creal(src[i]);
    if (im) im[i] = cimag(src[i]);
  }
}
static void join(real *dst, size_t n, const double *re, const double *im) {
  for (size_t i = 0; i < n; ++i) dst[i] = re[i] + I * (im ? im[i] : 0.0);
}
int or_cs_get_lattice(const or_sim *s, double *re, double *im) {
  split(s->fA, (size_t)9 * s->nx * s->ny, re, im);
  return OR_OK;
}
int or_cs_set_lattice(or_sim *s, const double *re, const double *im) {
  join(s->fA, (size_t)9 * s->nx * s->ny, re, im);
  return OR_OK;
}
int or_cs_get_mesh(const or_sim *s, double *re, double *im) {
  if (!s->m) return OR_E_STATE;
  split(s->fu, (size_t)9 * s->m->nnode, re, im);
  return OR_OK;
}
int or_cs_set_mesh(or_sim *s, const double *re, const double *im) {
  if (!s->m) return OR_E_STATE;
  join(s->fu, (size_t)9 * s->m->nnode, re, im);
  return OR_OK;
}
int64_t or_cs_history(const or_sim *s, double *re, double *im, int64_t cap) {
  const int64_t n = s->hist_n < cap ? s->hist_n : cap;
  split(s->hist, (size_t)2 * n, re, im);
  return s->hist_n;
}
#endif

/* Single-harmonic least-squares fit F(t) = F0 sin(omega t + phi) with omega
 * given, over the window [t0, t1) periods (the paper discards the first cycle
 * and uses three: [1, 4)), written as F = a_s sin + a_c cos; by
 * Eq.(force_phasor) F0 e^{i phi} = a_s + i a_c = (pi/4) rho omega^2 L^2 Theta A. */
int or_fit_theta(const double *hist, int64_t n, double omega, double A,
                 double b, double t0, double t1, double theta[2]) {
  if (!(omega > 0.0) || !(A != 0.0) || !(b > 0.0)) return OR_E_ARG;
  const double T = 2.0 * M_PI / omega;
  double ss = 0.0, sc = 0.0, cc = 0.0, sf = 0.0, cf = 0.0;
  int64_t cnt = 0;
  for (int64_t k = 0; k < n; ++k) {
    const double t = (double)(k + 1);
    if (t < t0 * T || t >= t1 * T) continue;
    const double sn = sin(omega * t), cs = cos(omega * t), F = hist[2 * k + 1];
    ss += sn * sn;
    sc += sn * cs;
    cc += cs * cs;
    sf += sn * F;
    cf += cs * F;
    ++cnt;
  }
  if (cnt < 2) return OR_E_ARG;
  const double det = ss * cc - sc * sc;
  if (!(fabs(det) > 0.0)) return OR_E_ARG;
  const double as = (sf * cc - cf * sc) / det;
  const double ac = (cf * ss - sf * sc) / det;
  const double norm = 0.25 * M_PI * 1.0 * omega * omega * b * b * A;
  theta[0] = as / norm;
  theta[1] = ac / norm;
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Structured refinement levels                                        */
/* ------------------------------------------------------------------ */
/* The paper splits the structured domain into refinement levels (Sec.
 * Problem statement, four levels, relaxation time given at the finest) but
 * prints no interface scheme. Reading taken: nested levels with a
 * refinement ratio of 2 and coinciding nodes, each level advancing with its
 * own Delta t = Delta x (acoustic scaling), so a level takes two steps per
 * step of the next coarser one. The viscosity is the same on every level:
 * with nu = c_s^2 (tau - 1/2) Delta x^2 / Delta t, tau_fine - 1/2 =
 * 2 (tau_coarse - 1/2). Level l+1 covers the node box [x0, x1] x [y0, y1] of
 * level l; its outermost ring of nodes lies on the box perimeter and is
 * written from level l before each of its steps, and level l's nodes one
 * inside the box are written from level l+1 after every second fine step
 * (the interface exchange of Dupuis and Chopard, Phys. Rev. E 67, 066707,
 * 2003, restated here from the Chapman-Enskog expansion):
 *   - the exchanged quantities are the pre-collision density, velocity and
 *     non-equilibrium part f - f^eq, as in the hybrid interfaces;
 *   - to first order f^neq = -tau rho w_i Q_i : grad u / c_s^2 with the
 *     gradient in the level's own lattice units, so f^neq scales with
 *     tau Delta x: fine = coarse * tau_f / (2 tau_c), and the inverse factor
 *     going the other way;
 *   - the written value is post-collision: f^eq + (1 - 1/tau) f^neq;
 *   - on the fine ring between two coarse nodes the quantities are linear
 *     in space; at the intermediate fine time they are linear in time
 *     between the coarse states at t and t + 1.
 * The finest level is a hybrid case (lattice plus body-fitted grid) in its
 * own lattice units, or a plain lattice without a grid. */
#ifndef OR_COMPLEX_STEP
typedef struct or_level {
  int nx, ny, bc;
  double tau;
  double *fA, *fB;           /* [9][ny][nx]: post-collision at t and t - 1 */
  int bx0, by0, bx1, by1;    /* node box of the next finer level           */
  double *m0, *m1;           /* [ny][nx][12] (rho, ux, uy, f^neq) at t, t+1,
                                filled on the box perimeter only           */
  double u_bot, u_top;       /* wall x-velocities (bc 0, coarsest level)   */
} or_level;

struct or_ml {
  int L;
  or_level lev[OR_ML_MAX_LEVELS]; /* levels 0 .. L-2 */
  or_sim *fine;                   /* level L-1       */
  int flags;
  int64_t k;                      /* steps of level 0 */
};

/* uniform view of a level's lattice (the finest lives in its or_sim) */
typedef struct { int nx, ny, bc; double tau; double *fA, *fB; } lview;

static lview level_view(const or_ml *s, int l) {
  lview v;
  if (l == s->L - 1) {
    v.nx = s->fine->nx; v.ny = s->fine->ny; v.bc = s->fine->bc;
    v.tau = s->fine->tau_s; v.fA = s->fine->fA; v.fB = s->fine->fB;
  } else {
    const or_level *c = &s->lev[l];
    v.nx = c->nx; v.ny = c->ny; v.bc = c->bc; v.tau = c->tau; v.fA = c->fA; v.fB = c->fB;
  }
  return v;
}

static int on_box_perimeter(const or_level *c, int x, int y) {
  if (x < c->bx0 || x > c->bx1 || y < c->by0 || y > c->by1) return 0;
  return x == c->bx0 || x == c->bx1 || y == c->by0 || y == c->by1;
}

/* Eq.(LBE) on a coarse level: every node except those strictly inside the
 * finer level's box (nobody reads them: the ones next to the perimeter are
 * written from the finer level) and, on a ring-fed level, its own ring. */
static void level_collide(or_level *c) {
  for (int y = 0; y < c->ny; ++y)
    for (int x = 0; x < c->nx; ++x) {
      if (x > c->bx0 && x < c->bx1 && y > c->by0 && y < c->by1) continue;
      if (c->bc == OR_BC_RING && (x == 0 || y == 0 || x == c->nx - 1 || y == c->ny - 1)) continue;
      double f[9], e[9], rho, ux, uy;
      pull_node(c->fA, c->nx, c->ny, c->bc, x, y, c->u_bot, c->u_top, f);
      moments(f, &rho, &ux, &uy);
      feq_r(rho, ux, uy, e);
      for (int i = 0; i < 9; ++i) c->fB[lidx(c->nx, c->ny, i, x, y)] = f[i] - (1.0 / c->tau) * (f[i] - e[i]);
    }
}

/* pre-collision moments at the box perimeter, pulled from post-collision
 * buffer P: the state one step after P */
static void box_moments(const or_level *c, const double *P, double *m) {
  for (int y = c->by0; y <= c->by1; ++y)
    for (int x = c->bx0; x <= c->bx1; ++x) {
      if (!on_box_perimeter(c, x, y)) continue;
      double f[9], e[9], rho, ux, uy;
      pull_node(P, c->nx, c->ny, c->bc, x, y, c->u_bot, c->u_top, f);
      moments(f, &rho, &ux, &uy);
      feq_r(rho, ux, uy, e);
      double *o = m + ((size_t)y * c->nx + x) * 12;
      o[0] = rho;
      o[1] = ux;
      o[2] = uy;
      for (int i = 0; i < 9; ++i) o[3 + i] = f[i] - e[i];
    }
}

/* Ring of level l+1 at its step h (0: time t of level l, 1: t + 1/2). */
static void prolong(or_ml *s, int l, int h) {
  const or_level *c = &s->lev[l];
  const lview f = level_view(s, l + 1);
  const double tw1 = 0.5 * (double)h, tw0 = 1.0 - tw1; /* weights of t, t+1 */
  const double rescale = (s->flags & OR_ML_FLAG_PLANT_NO_RESCALE) ? 1.0 : f.tau / (2.0 * c->tau);
  for (int j = 0; j < f.ny; ++j)
    for (int i = 0; i < f.nx; ++i) {
      if (!(i == 0 || j == 0 || i == f.nx - 1 || j == f.ny - 1)) continue;
      /* coarse position (bx0 + i/2, by0 + j/2): one node, or the midpoint of
       * two along the perimeter */
      const int X2 = 2 * c->bx0 + i, Y2 = 2 * c->by0 + j;
      int xa = X2 / 2, ya = Y2 / 2, xb = xa, yb = ya;
      if (X2 & 1) xb = xa + 1;
      if (Y2 & 1) yb = ya + 1;
      double q[12];
      for (int r = 0; r < 12; ++r) {
        const double *a0 = c->m0 + ((size_t)ya * c->nx + xa) * 12, *b0 = c->m0 + ((size_t)yb * c->nx + xb) * 12;
        const double *a1 = c->m1 + ((size_t)ya * c->nx + xa) * 12, *b1 = c->m1 + ((size_t)yb * c->nx + xb) * 12;
        q[r] = tw0 * 0.5 * (a0[r] + b0[r]) + tw1 * 0.5 * (a1[r] + b1[r]);
      }
      double e[9];
      feq_r(q[0], q[1], q[2], e);
      for (int k = 0; k < 9; ++k)
        f.fA[lidx(f.nx, f.ny, k, i, j)] = e[k] + (1.0 - 1.0 / f.tau) * rescale * q[3 + k];
    }
}

/* Level l's nodes one inside the box, from level l+1 at the common time:
 * the fine pre-collision state is pulled from the fine buffer one fine step
 * back. */
static void restrict_level(or_ml *s, int l) {
  or_level *c = &s->lev[l];
  const lview f = level_view(s, l + 1);
  const double rescale = (s->flags & OR_ML_FLAG_PLANT_NO_RESCALE) ? 1.0 : 2.0 * c->tau / f.tau;
  for (int y = c->by0 + 1; y <= c->by1 - 1; ++y)
    for (int x = c->bx0 + 1; x <= c->bx1 - 1; ++x) {
      if (!(x == c->bx0 + 1 || x == c->bx1 - 1 || y == c->by0 + 1 || y == c->by1 - 1)) continue;
      double g[9], e[9], rho, ux, uy;
      pull_node(f.fB, f.nx, f.ny, f.bc, 2 * (x - c->bx0), 2 * (y - c->by0), 0.0, 0.0, g);
      moments(g, &rho, &ux, &uy);
      feq_r(rho, ux, uy, e);
      for (int i = 0; i < 9; ++i)
        c->fA[lidx(c->nx, c->ny, i, x, y)] = e[i] + (1.0 - 1.0 / c->tau) * rescale * (g[i] - e[i]);
    }
}

/* one step of level l (and, recursively, two of each finer level) */
static int ml_advance(or_ml *s, int l) {
  if (l == s->L - 1) return or_step(s->fine, 1);
  or_level *c = &s->lev[l];
  /* 1. Eq.(LBE) on this level */
  level_collide(c);
  double *t = c->fA;
  c->fA = c->fB;
  c->fB = t;
  /* 2. perimeter moments at t + 1 */
  box_moments(c, c->fB, c->m1);
  /* 3. two steps of the finer level, its ring from this level at t, t + 1/2 */
  for (int h = 0; h < 2; ++h) {
    prolong(s, l, h);
    const int rc = ml_advance(s, l + 1);
    if (rc != OR_OK) return rc;
  }
  /* 4. the nodes one inside the box from the finer level at t + 1 */
  restrict_level(s, l);
  t = c->m0;
  c->m0 = c->m1;
  c->m1 = t;
  return OR_OK;
}

void or_ml_destroy(or_ml *s) {
  if (!s) return;
  for (int l = 0; l < s->L - 1; ++l) {
    free(s->lev[l].fA); free(s->lev[l].fB); free(s->lev[l].m0); free(s->lev[l].m1);
  }
  or_destroy(s->fine);
  free(s);
}

int or_ml_create(const or_config *fine, int32_t nlevels, int32_t nx0, int32_t ny0, int32_t bc0,
                 double u_bot, double u_top, const int32_t *box, int32_t flags, or_ml **out) {
  if (!fine || !box || !out) return OR_E_ARG;
  *out = NULL;
  if (nlevels < 2 || nlevels > OR_ML_MAX_LEVELS) return OR_E_ARG;
  if (bc0 != OR_BC_PERIODIC_X_WALLS_Y && bc0 != OR_BC_PERIODIC && bc0 != OR_BC_PAPER) return OR_E_ARG;
  if (bc0 != OR_BC_PERIODIC_X_WALLS_Y && (u_bot != 0.0 || u_top != 0.0)) return OR_E_ARG;
  if (fine->bc != OR_BC_RING || !(fine->tau > 0.5)) return OR_E_ARG;
  or_ml *s = xcalloc(1, sizeof(or_ml));
  if (!s) return OR_E_NOMEM;
  s->L = nlevels;
  s->flags = flags;
  /* level sizes from the boxes, relaxation times from the finest down */
  int nx = nx0, ny = ny0;
  for (int l = 0; l < nlevels - 1; ++l) {
    or_level *c = &s->lev[l];
    c->nx = nx;
    c->ny = ny;
    c->bc = l == 0 ? bc0 : OR_BC_RING;
    c->u_bot = l == 0 ? u_bot : 0.0;
    c->u_top = l == 0 ? u_top : 0.0;
    c->bx0 = box[4 * l];
    c->by0 = box[4 * l + 1];
    c->bx1 = box[4 * l + 2];
    c->by1 = box[4 * l + 3];
    if (nx < 3 || ny < 3 || c->bx0 < 2 || c->by0 < 2 || c->bx1 > nx - 3 || c->by1 > ny - 3 ||
        c->bx1 - c->bx0 < 4 || c->by1 - c->by0 < 4) {
      or_ml_destroy(s);
      return OR_E_ARG;
    }
    nx = 2 * (c->bx1 - c->bx0) + 1;
    ny = 2 * (c->by1 - c->by0) + 1;
  }
  if (fine->nx != nx || fine->ny != ny) {
    or_ml_destroy(s);
    return OR_E_ARG;
  }
  double tau = fine->tau;
  for (int l = nlevels - 2; l >= 0; --l) {
    tau = 0.5 + 0.5 * (tau - 0.5);
    if (s->flags & OR_ML_FLAG_PLANT_SAME_TAU) tau = fine->tau;
    s->lev[l].tau = tau;
  }
  const int rc = or_create(fine, &s->fine);
  if (rc != OR_OK) {
    or_ml_destroy(s);
    return rc;
  }
  for (int l = 0; l < nlevels - 1; ++l) {
    or_level *c = &s->lev[l];
    const size_t n = (size_t)c->nx * c->ny;
    c->fA = malloc(9 * n * sizeof(double));
    c->fB = malloc(9 * n * sizeof(double));
    c->m0 = xcalloc(12 * n, sizeof(double));
    c->m1 = xcalloc(12 * n, sizeof(double));
    if (!c->fA || !c->fB || !c->m0 || !c->m1) {
      or_ml_destroy(s);
      return OR_E_NOMEM;
    }
    /* at rest with unit density, like the finest level */
    for (int i = 0; i < 9; ++i)
      for (size_t p = 0; p < n; ++p) c->fA[(size_t)i * n + p] = c->fB[(size_t)i * n + p] = WT[i];
    box_moments(c, c->fA, c->m0);
  }
  *out = s;
  return OR_OK;
}

int or_ml_step(or_ml *s, int64_t nsteps) {
  if (!s || nsteps < 0) return OR_E_ARG;
  const int64_t per = (int64_t)1 << (s->L - 1);
  if (s->fine->m && s->fine->hist_n + nsteps * per > s->fine->hist_cap) return OR_E_ARG;
  for (int64_t it = 0; it < nsteps; ++it) {
    const int rc = ml_advance(s, 0);
    if (rc != OR_OK) return rc;
    s->k++;
  }
  return OR_OK;
}

int or_ml_level_shape(const or_ml *s, int32_t level, int32_t *nx, int32_t *ny, double *tau) {
  if (!s || level < 0 || level >= s->L) return OR_E_ARG;
  const lview v = level_view(s, level);
  if (nx) *nx = v.nx;
  if (ny) *ny = v.ny;
  if (tau) *tau = v.tau;
  return OR_OK;
}

int or_ml_get_level(const or_ml *s, int32_t level, double *out) {
  if (!s || !out || level < 0 || level >= s->L) return OR_E_ARG;
  const lview v = level_view(s, level);
  memcpy(out, v.fA, (size_t)9 * v.nx * v.ny * sizeof(double));
  return OR_OK;
}

/* Sets level `level` to a state taken as steady: both of its buffers get
 * it, and the moments on the perimeter of the finer level's box are
 * recomputed from it as those of the current time. */
int or_ml_set_level(or_ml *s, int32_t level, const double *in) {
  if (!s || !in || level < 0 || level >= s->L) return OR_E_ARG;
  const lview v = level_view(s, level);
  const size_t bytes = (size_t)9 * v.nx * v.ny * sizeof(double);
  memcpy(v.fA, in, bytes);
  memcpy(v.fB, in, bytes);
  if (level < s->L - 1) box_moments(&s->lev[level], s->lev[level].fA, s->lev[level].m0);
  return OR_OK;
}

or_sim *or_ml_finest(or_ml *s) { return s ? s->fine : NULL; }
int64_t or_ml_steps(const or_ml *s) { return s ? s->k : 0; }
#endif
