/*
 * sanitize_main.c -- drives every entry point of the CPU oracle on small
 * cases, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitize.py builds and runs it). TEST INFRASTRUCTURE:
 * it checks the oracle's memory and arithmetic hygiene, not its results.
 * Built a second time with -DOR_COMPLEX_STEP it drives the complex-step
 * variant. Exit status 0 when every call returned as expected.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hlbm_oracle.h"

#ifdef OR_COMPLEX_STEP
/* entry points of the complex-step build only */
int or_cs_perturb(or_sim *s, double hA, double homega, double htau);
int or_cs_get_lattice(const or_sim *s, double *re, double *im);
int or_cs_set_lattice(or_sim *s, const double *re, const double *im);
int64_t or_cs_history(const or_sim *s, double *re, double *im, int64_t cap);
#endif

static int failures = 0;
#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

static or_config lamina(int nx, int ny, int nux, int nuy, double h, double b, double tau, int flags, int steps) {
  or_config c;
  memset(&c, 0, sizeof(c));
  c.nx = nx;
  c.ny = ny;
  c.nux = nux;
  c.nuy = nuy;
  c.h_u = h;
  c.b = b;
  c.thickness = h;
  c.tau = tau;
  c.kc = 1.0;
  c.beta = 20.0;
  c.bc = OR_BC_PERIODIC_X_WALLS_Y;
  c.flags = flags;
  c.max_steps = steps;
  return c;
}

static void run_case(or_config c, int steps) {
  or_sim *s = NULL;
  EXPECT(or_create(&c, &s) == OR_OK);
  if (!s) return;
  EXPECT(or_step(s, steps) == OR_OK);
  or_info inf;
  EXPECT(or_info_get(s, &inf) == OR_OK);
#ifndef OR_COMPLEX_STEP
  double *buf = malloc(sizeof(double) * 9 * (size_t)c.nx * c.ny);
  EXPECT(or_get_lattice(s, buf) == OR_OK);
  EXPECT(or_set_lattice(s, buf) == OR_OK);
  free(buf);
  if (inf.nnode > 0) {
    double *g = malloc(sizeof(double) * 9 * (size_t)inf.nnode);
    EXPECT(or_get_mesh(s, g) == OR_OK);
    EXPECT(or_set_mesh(s, g) == OR_OK);
    free(g);
    double *h = malloc(sizeof(double) * 2 * (size_t)steps);
    EXPECT(or_history(s, h, steps) == steps);
    double th[2];
    (void)or_fit_theta(h, steps, inf.omega, inf.A, c.b, 0.0, 1.0, th);
    free(h);
    double p[12];
    EXPECT(or_probe_bilinear(s, 0.5 * c.nx + 0.25, 0.5 * c.ny + 0.75, p) == OR_OK);
    (void)or_probe_grid(s, 0.5 * c.nx + 0.3, 0.5 * (c.ny - 1) + 0.4, p);
    (void)or_lattice_status(s, steps, c.nx / 2, c.ny / 2);
  }
#else
  double *re = malloc(sizeof(double) * 9 * (size_t)c.nx * c.ny), *im = malloc(sizeof(double) * 9 * (size_t)c.nx * c.ny);
  EXPECT(or_cs_get_lattice(s, re, im) == OR_OK);
  EXPECT(or_cs_set_lattice(s, re, im) == OR_OK);
  free(re);
  free(im);
#endif
  or_destroy(s);
}

int main(void) {
  /* lattice alone, every boundary type */
  for (int bc = 0; bc <= 2; ++bc) {
    or_config c = lamina(12, 9, 0, 0, 1.0, 0.0, 0.8, 0, 4);
    c.bc = bc;
    run_case(c, 4);
  }
  /* lamina cases: uniform, odd width, no body, type-2 refills (fine grid) */
  run_case(lamina(64, 48, 24, 16, 1.0, 8.0, 0.8, 0, 12), 12);
  run_case(lamina(77, 45, 33, 16, 1.0, 9.0, 0.7, 0, 10), 10);
  run_case(lamina(64, 48, 24, 16, 1.0, 8.0, 0.8, OR_FLAG_NO_BODY | OR_FLAG_PLANT_S_FACTOR | OR_FLAG_PLANT_BARY, 8), 8);
  {
    or_config c = lamina(48, 48, 90, 44, 0.2, 8.0, 0.8, 0, 6);
    c.kc = 1.8;
    c.beta = 10.0;
    c.n_sub = 32;
    run_case(c, 6);
  }
#ifndef OR_COMPLEX_STEP
  /* meshes and their matrices */
  or_mesh *ms[3] = {or_mesh_lamina(10, 8, 1.0, 3.0), or_mesh_periodic(6, 5, 1.0), or_mesh_channel(5, 6, 1.0)};
  for (int i = 0; i < 3; ++i) {
    or_mesh *m = ms[i];
    EXPECT(m != NULL);
    if (!m) continue;
    const int n = or_mesh_nnode(m), k = or_mesh_kmax(m), t = or_mesh_ntri(m);
    double *x = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * n);
    int32_t *ty = malloc(sizeof(int32_t) * n), *nbr = malloc(sizeof(int32_t) * n * k), *tri = malloc(sizeof(int32_t) * 3 * t);
    double *S = malloc(sizeof(double) * n * 9 * k), *C = malloc(sizeof(double) * n * k), *V = malloc(sizeof(double) * n);
    double *txy = malloc(sizeof(double) * 6 * t), *f = malloc(sizeof(double) * 9 * n), *g = malloc(sizeof(double) * 9 * n);
    double *u = calloc(n, sizeof(double));
    or_mesh_nodes(m, x, y, ty);
    or_mesh_triangles(m, tri, txy);
    or_mesh_stencil(m, k, nbr, S, C, V);
    double lam[3];
    (void)or_mesh_locate(m, x[0] + 0.3, y[0] + 0.2, lam);
    for (int j = 0; j < 9 * n; ++j) f[j] = 1.0 / 9.0;
    or_fv_substep(m, f, f, g, g, 0.3, 0.25, u, u);
    double F[2];
    or_mesh_force(m, g, F);
    free(x); free(y); free(ty); free(nbr); free(tri); free(S); free(C); free(V); free(txy); free(f); free(g); free(u);
    or_mesh_free(m);
  }
  /* graded grid */
  {
    double X[14], Y[12];
    for (int i = 0; i < 14; ++i) X[i] = -7.0 + i + 0.01 * i * i;
    const double Yh[6] = {0.5, 1.5, 2.6, 3.8, 5.2, 6.8};
    for (int j = 0; j < 6; ++j) {
      Y[6 + j] = Yh[j];
      Y[5 - j] = -Yh[j];
    }
    or_config c = lamina(64, 48, 14, 12, 1.0, 4.0, 0.8, 0, 5);
    c.thickness = 1.0;
    or_sim *s = NULL;
    EXPECT(or_create_graded(&c, X, Y, &s) == OR_OK);
    if (s) {
      EXPECT(or_step(s, 5) == OR_OK);
      or_destroy(s);
    }
  }
  /* coupled motion */
  {
    or_config c = lamina(64, 48, 24, 16, 1.0, 8.0, 0.8, 0, 6);
    or_sim *s = NULL;
    EXPECT(or_create(&c, &s) == OR_OK);
    if (s) {
      EXPECT(or_set_motion(s, 50.0, 0.01, 0.0, 0.2, 0.0, 2.0) == OR_OK);
      EXPECT(or_step(s, 6) == OR_OK);
      double mh[12];
      EXPECT(or_motion_history(s, mh, 6) == 6);
      or_destroy(s);
    }
  }
  /* grid band on a moving wall, moving lattice walls */
  {
    or_config c = lamina(8, 24, 0, 0, 1.0, 0.0, 0.8, OR_FLAG_PLANT_NO_KNEQ, 6);
    or_sim *s = NULL;
    EXPECT(or_create_wallband(&c, 6, 0.4, 0.3, 0.01, 0.05, &s) == OR_OK);
    if (s) {
      EXPECT(or_set_walls(s, 0.0, 0.001) == OR_OK);
      EXPECT(or_step(s, 6) == OR_OK);
      or_destroy(s);
    }
  }
  /* a given triangulation: a 13 x 12 node grid with jittered interior
   * nodes, cells split along alternating diagonals, a lamina hole */
  {
    enum { NX = 13, NY = 12 };
    double xy[2 * NX * NY];
    int32_t ty[NX * NY], tri[3 * 2 * (NX - 1) * (NY - 1)];
    for (int j = 0; j < NY; ++j)
      for (int i = 0; i < NX; ++i) {
        const int p = j * NX + i;
        const int outer = i == 0 || j == 0 || i == NX - 1 || j == NY - 1;
        const int wall = (j == NY / 2 - 1 || j == NY / 2) && i >= 4 && i <= 8;
        xy[2 * p] = (i - 6) + (outer || wall ? 0.0 : 0.13 * ((i * 7 + j * 3) % 5 - 2) / 2.0);
        xy[2 * p + 1] = (j - 0.5 * (NY - 1)) + (outer || wall ? 0.0 : 0.11 * ((i * 5 + j * 11) % 5 - 2) / 2.0);
        ty[p] = wall ? OR_NODE_WALL : outer ? OR_NODE_INTERFACE : OR_NODE_INTERIOR;
      }
    int nt = 0;
    for (int cj = 0; cj + 1 < NY; ++cj)
      for (int ci = 0; ci + 1 < NX; ++ci) {
        if (cj == NY / 2 - 1 && ci >= 4 && ci < 8) continue; /* the lamina, x in [-2, 2], y in [-0.5, 0.5] */
        const int n00 = cj * NX + ci, n10 = n00 + 1, n01 = n00 + NX, n11 = n01 + 1;
        if ((ci + cj) % 2) {
          const int t[6] = {n00, n10, n11, n00, n11, n01};
          memcpy(&tri[3 * nt], t, sizeof(t));
        } else {
          const int t[6] = {n00, n10, n01, n10, n11, n01};
          memcpy(&tri[3 * nt], t, sizeof(t));
        }
        nt += 2;
      }
    or_config c = lamina(40, 30, 0, 0, 1.0, 4.0, 0.8, 0, 6);
    or_sim *s = NULL;
    EXPECT(or_create_mesh(&c, NX * NY, xy, ty, nt, tri, &s) == OR_OK);
    if (s) {
      EXPECT(or_step(s, 6) == OR_OK);
      EXPECT(or_set_deformation(s, 0.2, 0.0) == OR_E_ARG); /* after the first step */
      or_destroy(s);
    }
    /* the same grid bending with the lamina */
    EXPECT(or_create_mesh(&c, NX * NY, xy, ty, nt, tri, &s) == OR_OK);
    if (s) {
      EXPECT(or_set_deformation(s, 1.5, 0.0) == OR_E_ARG);
      EXPECT(or_set_deformation(s, 0.25, 0.4) == OR_OK);
      EXPECT(or_step(s, 6) == OR_OK);
      or_destroy(s);
    }
    tri[0] = NX * NY; /* out of range */
    EXPECT(or_create_mesh(&c, NX * NY, xy, ty, nt, tri, &s) == OR_E_ARG && s == NULL);
  }
  /* refinement levels */
  {
    or_config f = lamina(0, 0, 0, 0, 1.0, 0.0, 0.8, 0, 4);
    f.bc = OR_BC_RING;
    const int32_t box[4] = {4, 4, 12, 12};
    f.nx = 2 * (box[2] - box[0]) + 1;
    f.ny = 2 * (box[3] - box[1]) + 1;
    or_ml *s = NULL;
    EXPECT(or_ml_create(&f, 2, 17, 17, OR_BC_PERIODIC_X_WALLS_Y, 0.0, 0.001, box, 0, &s) == OR_OK);
    if (s) {
      EXPECT(or_ml_step(s, 3) == OR_OK);
      int32_t nx, ny;
      double tau;
      EXPECT(or_ml_level_shape(s, 0, &nx, &ny, &tau) == OR_OK);
      double *buf = malloc(sizeof(double) * 9 * nx * ny);
      EXPECT(or_ml_get_level(s, 0, buf) == OR_OK);
      EXPECT(or_ml_set_level(s, 0, buf) == OR_OK);
      free(buf);
      or_ml_destroy(s);
    }
  }
  /* rejected arguments */
  {
    or_config c = lamina(64, 48, 24, 16, 1.0, 8.0, 0.5, 0, 4);
    or_sim *s = NULL;
    EXPECT(or_create(&c, &s) != OR_OK && s == NULL);
  }
#else
  {
    or_config c = lamina(64, 48, 24, 16, 1.0, 8.0, 0.8, 0, 6);
    or_sim *s = NULL;
    EXPECT(or_create(&c, &s) == OR_OK);
    if (s) {
      EXPECT(or_cs_perturb(s, 1e-30, 0.0, 0.0) == OR_OK);
      EXPECT(or_step(s, 6) == OR_OK);
      double re[12], im[12];
      EXPECT(or_cs_history(s, re, im, 6) == 6);
      or_destroy(s);
    }
  }
#endif
  if (failures) fprintf(stderr, "%d expectation(s) failed\n", failures);
  else printf("sanitized oracle run: ok\n");
  return failures ? 1 : 0;
}
