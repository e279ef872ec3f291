// Device helpers shared by the forward and the adjoint kernels: D2Q9
// constants, storage traits, equilibrium and moments with their
// vector-Jacobian products, the streaming pull and its source addresses, and
// the interpolation geometry (lattice cells, grid triangles, refill types).
// Forward and adjoint take every discrete decision through the same code.
//
// D2Q9 ordering: rest, (1,0), (0,1), (-1,0), (0,-1), (1,1), (-1,1), (-1,-1),
// (1,-1); weights 4/9, 1/9 (axis), 1/36 (diagonal); c_s^2 = 1/3.
#pragma once

#include <cmath>

#include "hlbm_internal.h"

namespace mghlbm {
namespace dev {

constexpr int CXd[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CYd[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

template <class R>
__device__ __forceinline__ R wgt(int q) {
  return q == 0 ? R(4.0 / 9.0) : (q < 5 ? R(1.0 / 9.0) : R(1.0 / 36.0));
}

// ---- storage traits --------------------------------------------------------
template <class T>
struct Stor;
// st_stream: store of a value that is not read again in this kernel; the
// lattice output is streamed with non-temporal stores.
template <>
struct Stor<double> {
  static __device__ __forceinline__ double ld(const double *p, size_t i, int) { return p[i]; }
  static __device__ __forceinline__ void st(double *p, size_t i, int, double v) { p[i] = v; }
  static __device__ __forceinline__ void st_stream(double *p, size_t i, int, double v) {
    __builtin_nontemporal_store(v, p + i);
  }
  // the value a store followed by a load returns
  static __device__ __forceinline__ double round_trip(double v, int) { return v; }
};
template <>
struct Stor<float> {
  static __device__ __forceinline__ float ld(const float *p, size_t i, int) { return p[i]; }
  static __device__ __forceinline__ void st(float *p, size_t i, int, float v) { p[i] = v; }
  static __device__ __forceinline__ void st_stream(float *p, size_t i, int, float v) {
    __builtin_nontemporal_store(v, p + i);
  }
  static __device__ __forceinline__ float round_trip(float v, int) { return v; }
};
template <>
struct Stor<__half> {  // deviation from the rest equilibrium w_i
  static __device__ __forceinline__ float ld(const __half *p, size_t i, int q) {
    return __half2float(p[i]) + wgt<float>(q);
  }
  static __device__ __forceinline__ void st(__half *p, size_t i, int q, float v) {
    p[i] = __float2half_rn(v - wgt<float>(q));
  }
  static __device__ __forceinline__ void st_stream(__half *p, size_t i, int q, float v) {
    const __half h = __float2half_rn(v - wgt<float>(q));
    __builtin_nontemporal_store(*reinterpret_cast<const unsigned short *>(&h),
                                reinterpret_cast<unsigned short *>(p + i));
  }
  static __device__ __forceinline__ float round_trip(float v, int q) {
    return __half2float(__float2half_rn(v - wgt<float>(q))) + wgt<float>(q);
  }
};

// Fused multiply-add written out: the kernels are compiled without implicit
// contraction, so every fusion is explicit and rounds the same wherever the
// expression is inlined.
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// ---- D2Q9 equilibrium and moments ------------------------------------------
// Eq.(local_eq) with c_s^2 = 1/3: w rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2)
template <class R>
__device__ __forceinline__ void equilibrium(R rho, R ux, R uy, R e[9]) {
  const R one_uu = fmad(R(-1.5), fmad(ux, ux, uy * uy), R(1));
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const R cu = R(CXd[q]) * ux + R(CYd[q]) * uy;  // c components are 0 or +-1: exact
    e[q] = wgt<R>(q) * rho * fmad(R(4.5) * cu, cu, fmad(R(3), cu, one_uu));
  }
}

template <class R>
__device__ __forceinline__ void moments(const R f[9], R &rho, R &ux, R &uy) {
  rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const R mx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const R my = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  const R inv = R(1) / rho;
  ux = mx * inv;
  uy = my * inv;
}

// (a_rho, a_x, a_y) = (d f^eq / d(rho, u_x, u_y))^T g
template <class R>
__device__ __forceinline__ void equilibrium_vjp(R rho, R ux, R uy, const R g[9], R &ar, R &ax, R &ay) {
  const R uu = R(1.5) * (ux * ux + uy * uy);
  ar = ax = ay = R(0);
  R su = R(0);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const R cu = R(CXd[q]) * ux + R(CYd[q]) * uy;
    const R wg = wgt<R>(q) * g[q];
    ar += wg * (R(1) + R(3) * cu + R(4.5) * cu * cu - uu);
    const R d = wg * (R(3) + R(9) * cu);
    ax += R(CXd[q]) * d;
    ay += R(CYd[q]) * d;
    su += wg;
  }
  ax = rho * (ax - R(3) * ux * su);
  ay = rho * (ay - R(3) * uy * su);
}

// Adjoint of a node's interpolation inputs: given the cotangents (zr, zx, zy,
// zn[9]) of (rho, u_x, u_y, f^neq = f - f^eq(rho, u)) of the node's state f,
// returns fb = d/df of <z, (rho, u, f^neq)>.
template <class R>
__device__ __forceinline__ void node_chain(R rho, R ux, R uy, R zr, R zx, R zy, const R zn[9], R fb[9]) {
  R ar, ax, ay;
  equilibrium_vjp<R>(rho, ux, uy, zn, ar, ax, ay);
  const R inv = R(1) / rho;
  const R br = zr - ar, bx = (zx - ax) * inv, by = (zy - ay) * inv;
  const R base = br - bx * ux - by * uy;
#pragma unroll
  for (int q = 0; q < 9; ++q) fb[q] = zn[q] + base + bx * R(CXd[q]) + by * R(CYd[q]);
}

// ---- streaming ----------------------------------------------------------------
// Flat indices into a [9][plane] array (plane >= ny * nx, row-major nodes)
// of the nine values the pull of node (x, y) reads: population q arriving
// at (x, y) left x - c_q one step earlier. bc 0: periodic in x, and across a
// resting y wall halfway bounce-back returns the opposite population of the
// node itself; bc 1: periodic in x and y; bc 2 (the paper's boundaries):
// the same bounce-back across the x walls, and at a y end the incoming
// population equals that of the next row in (zero normal gradient), i.e. it
// is pulled from the node's own row; a population crossing both a wall and
// an end is reflected by the wall. For bc 0 and 1 every (population, node)
// pair of the array is the source of exactly one (q, node) pair, so the
// adjoint of the pull is a push to these same addresses (not so for bc 2).
__device__ __forceinline__ void pull_index(int nx, int ny, size_t plane, int bc, int x, int y, size_t idx[9]) {
  const int xm = x == 0 ? nx - 1 : x - 1;
  const int xp = x == nx - 1 ? 0 : x + 1;
  int ym = y - 1, yp = y + 1;
  bool lo = false, hi = false, wl = false, wr = false;
  if (bc == 1) {
    ym = y == 0 ? ny - 1 : ym;
    yp = y == ny - 1 ? 0 : yp;
  } else if (bc == 2) {
    ym = y == 0 ? y : ym;
    yp = y == ny - 1 ? y : yp;
    wl = (x == 0);
    wr = (x == nx - 1);
  } else {
    lo = (y == 0);
    hi = (y == ny - 1);
  }
  const size_t r = (size_t)y * nx, rm = (size_t)ym * nx, rp = (size_t)yp * nx;
  const size_t c = r + x;
  idx[0] = c;
  idx[1] = wl ? 3 * plane + c : 1 * plane + r + xm;
  idx[3] = wr ? 1 * plane + c : 3 * plane + r + xp;
  idx[2] = lo ? 4 * plane + c : 2 * plane + rm + x;
  idx[5] = wl ? 7 * plane + c : (lo ? 7 * plane + c : 5 * plane + rm + xm);
  idx[6] = wr ? 8 * plane + c : (lo ? 8 * plane + c : 6 * plane + rm + xp);
  idx[4] = hi ? 2 * plane + c : 4 * plane + rp + x;
  idx[7] = wr ? 5 * plane + c : (hi ? 5 * plane + c : 7 * plane + rp + xp);
  idx[8] = wl ? 6 * plane + c : (hi ? 6 * plane + c : 8 * plane + rp + xm);
}

// The same streaming rules as pull_index, as the source of one population:
// population q arriving at (x, y) is population qs of node (xs, ys) one step
// earlier (bc 0, 1, 2).
__device__ __forceinline__ void pull_source(int nx, int ny, int bc, int x, int y, int q, int &qs, int &xs,
                                            int &ys) {
  constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  int sx = x - CXd[q], sy = y - CYd[q];
  qs = q;
  if (bc == 2) {
    if (sx < 0 || sx >= nx) {  // x wall: halfway bounce-back, also at the corners
      qs = opp[q];
      xs = x;
      ys = y;
      return;
    }
    if (sy < 0 || sy >= ny) sy = y;  // y end: from the node's own row
    xs = sx;
    ys = sy;
    return;
  }
  xs = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
  if (bc == 1) {
    ys = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
    return;
  }
  if (sy < 0 || sy >= ny) {  // y wall: halfway bounce-back
    qs = opp[q];
    xs = x;
    ys = y;
    return;
  }
  ys = sy;
}

// Populations arriving at lattice node (x, y) at t_{k+1}: pulled from the
// post-collision buffer of t_k (left side of Eq.(LBE)).
template <class T, class R>
__device__ __forceinline__ void pull(const T *__restrict__ A, int nx, int ny, size_t plane, int bc, int x,
                                     int y, R f[9]) {
  size_t idx[9];
  pull_index(nx, ny, plane, bc, x, y, idx);
  // a bounced-back value comes from the opposite population, whose rest
  // weight w_i is the same
#pragma unroll
  for (int q = 0; q < 9; ++q) f[q] = Stor<T>::ld(A, idx[q], q);
}

// ---- interpolation geometry ---------------------------------------------------
// Lattice cell of point (X, Y) and the bilinear weight of its corner d (d & 1:
// x + 1, d >> 1: y + 1), with dw/dY (the grid moves in y only).
__device__ __forceinline__ void bilinear_corner(double X, double Y, int d, int &xd, int &yd, double &w,
                                                double &dw_dY) {
  const double fx = floor(X), fy = floor(Y);
  const double a = X - fx, b = Y - fy;
  const double wx = d & 1 ? a : 1.0 - a;
  w = wx * (d >> 1 ? b : 1.0 - b);
  dw_dY = d >> 1 ? wx : -wx;
  xd = (int)fx + (d & 1);
  yd = (int)fy + (d >> 1);
}

// Triangle of the grid cell (ci, cj) containing local cell coordinates
// (a, b) in [0,1]^2, its barycentric weights and their derivative in b.
// Cells left of the centre line are cut by the rising diagonal, cells right
// of it by the falling one. tri: 0 the cell's first triangle, 1 its second,
// -1 the one the coordinates fall in (the first on the diagonal).
__device__ __forceinline__ void cell_triangle(int ci, int cj, int nux, double a, double b, int node[3],
                                              double lam[3], double dlam_db[3], int tri = -1) {
  const int n00 = cj * nux + ci, n10 = n00 + 1, n01 = n00 + nux, n11 = n01 + 1;
  if (2 * ci + 1 < nux) {
    if (tri == 0 || (tri < 0 && b <= a)) {  // (n00, n10, n11)
      node[0] = n00; node[1] = n10; node[2] = n11;
      lam[0] = 1.0 - a; lam[1] = a - b; lam[2] = b;
      dlam_db[0] = 0.0; dlam_db[1] = -1.0; dlam_db[2] = 1.0;
    } else {       // (n00, n11, n01)
      node[0] = n00; node[1] = n11; node[2] = n01;
      lam[0] = 1.0 - b; lam[1] = a; lam[2] = b - a;
      dlam_db[0] = -1.0; dlam_db[1] = 0.0; dlam_db[2] = 1.0;
    }
  } else {
    if (tri == 0 || (tri < 0 && a + b <= 1.0)) {  // (n00, n10, n01)
      node[0] = n00; node[1] = n10; node[2] = n01;
      lam[0] = 1.0 - a - b; lam[1] = a; lam[2] = b;
      dlam_db[0] = -1.0; dlam_db[1] = 0.0; dlam_db[2] = 1.0;
    } else {             // (n10, n11, n01)
      node[0] = n10; node[1] = n11; node[2] = n01;
      lam[0] = 1.0 - b; lam[1] = a + b - 1.0; lam[2] = 1.0 - a;
      dlam_db[0] = -1.0; dlam_db[1] = 1.0; dlam_db[2] = 0.0;
    }
  }
}

// Point location on an unstructured grid: the lowest-numbered triangle that
// holds (px, py) (local frame) with every barycentric coordinate >= -1e-12,
// or -1. The bucket of the point lists, in increasing order, every triangle
// that can hold it. Each coordinate is the signed area of the sub-triangle
// opposite its vertex over the triangle's.

__device__ __forceinline__ double edge_area(double ax, double ay, double bx, double by, double px, double py) {
  return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

__device__ inline int mesh_locate(const MeshGeom &m, double px, double py, int node[3], double lam[3]) {
  const int bi = (int)floor((px - m.bx0) / kBucket), bj = (int)floor((py - m.by0) / kBucket);
  if (bi < 0 || bj < 0 || bi >= m.bnx || bj >= m.bny) return -1;
  const int b = bj * m.bnx + bi;
  for (int s = m.bstart[b]; s < m.bstart[b + 1]; ++s) {
    const int t = m.blist[s];
    const double *q = m.txy + 6 * (size_t)t;
    const double D = edge_area(q[0], q[1], q[2], q[3], q[4], q[5]);
    const double l0 = edge_area(q[2], q[3], q[4], q[5], px, py) / D;
    const double l1 = edge_area(q[4], q[5], q[0], q[1], px, py) / D;
    const double l2 = edge_area(q[0], q[1], q[2], q[3], px, py) / D;
    if (l0 >= -1e-12 && l1 >= -1e-12 && l2 >= -1e-12) {
      lam[0] = l0;
      lam[1] = l1;
      lam[2] = l2;
      for (int a = 0; a < 3; ++a) node[a] = m.tri[3 * (size_t)t + a];
      return t;
    }
  }
  return -1;
}

// Grid geometry needed to place nodes and classify refills.
struct GridGeom {
  int nux, nuy;
  double h, xc, half_b, half_T;
  int body;
  // graded grid: local x of every column, y of every row (null: uniform
  // spacing h, column i at (i - nux/2) h, row j at (j - (nuy-1)/2) h)
  const double *gx = nullptr, *gy = nullptr;
};

// largest c in [0, n-2] with v[c] <= x (0 when x < v[0]); v increasing
__device__ __forceinline__ int graded_cell(const double *v, int n, double x) {
  int lo = 0, hi = n - 2;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (v[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// true for a cell of the lamina slot (no triangles)
__device__ __forceinline__ bool body_cell(const GridGeom &g, int ci, int cj) {
  if (!g.body || cj != g.nuy / 2 - 1) return false;
  if (g.gx) {
    const double half = g.half_b + 1e-9 * (2.0 * g.half_T);
    return g.gx[ci] >= -half && g.gx[ci + 1] <= half;
  }
  const double half = g.half_b + 1e-9 * g.h;
  return (double)(ci - g.nux / 2) * g.h >= -half && (double)(ci + 1 - g.nux / 2) * g.h <= half;
}

// whether triangle tri (0: the cell's first) of cell ci holds local
// coordinates (a, b), every barycentric weight >= -tol
__device__ __forceinline__ bool cell_holds(int ci, int nux, double a, double b, int tri, double tol) {
  if (2 * ci + 1 < nux) {
    if (tri == 0) return 1.0 - a >= -tol && a - b >= -tol && b >= -tol;
    return 1.0 - b >= -tol && a >= -tol && b - a >= -tol;
  }
  if (tri == 0) return 1.0 - a - b >= -tol && a >= -tol && b >= -tol;
  return 1.0 - b >= -tol && a + b - 1.0 >= -tol && 1.0 - a >= -tol;
}

// Point location with the tie rule of the reading: a point goes to the
// lowest-numbered triangle that holds it within 1e-12 in its barycentric
// weights, triangles numbered cell by cell row-major from the bottom row,
// a cell's first triangle first. The point lies in or next to cell
// (ci0, cj0); coord(i, j, a, b) gives its local coordinates in cell (i, j).
// Only where several triangles hold the point does the choice matter, and
// then only for derivatives across a row line (values are continuous).
template <class Coord>
__device__ __forceinline__ bool lowest_triangle(const GridGeom &g, int ci0, int cj0, Coord coord, int &ci, int &cj,
                                                double &a, double &b, int &tri) {
  const double tol = 1e-12;
  // the neighbours below, left of, right of or above cell (ci0, cj0) can
  // hold the point only when it lies within tol of that side
  double a0, b0;
  coord(ci0, cj0, a0, b0);
  const int jlo = b0 <= tol ? -1 : 0, jhi = b0 >= 1.0 - tol ? 1 : 0;
  const int ilo = a0 <= tol ? -1 : 0, ihi = a0 >= 1.0 - tol ? 1 : 0;
  for (int dj = jlo; dj <= jhi; ++dj)
    for (int di = ilo; di <= ihi; ++di) {
      const int i = ci0 + di, j = cj0 + dj;
      if (i < 0 || j < 0 || i > g.nux - 2 || j > g.nuy - 2) continue;
      double aa, bb;
      coord(i, j, aa, bb);
      // outside the cell's closed square widened by tol: no triangle of it
      if (aa < -tol || aa > 1.0 + tol || bb < -tol || bb > 1.0 + tol || body_cell(g, i, j)) continue;
      for (int t = 0; t < 2; ++t)
        if (cell_holds(i, g.nux, aa, bb, t, tol)) {
          ci = i;
          cj = j;
          a = aa;
          b = bb;
          tri = t;
          return true;
        }
    }
  return false;
}

// Lattice node (x, y) inside the grid at t_k (lower grid row at Y0): its
// cell, local coordinates and triangle, as used by the lattice
// interpolation nodes.
__device__ __forceinline__ void lattice_node_cell(const GridGeom &g, double ybase, int x, int y, int &ci, int &cj,
                                                  double &a, double &b, int &tri) {
  tri = -1;
  if (g.gx) {  // graded: the cell holding the point, local coordinates in [0, 1]
    const double lx = (double)x - g.xc, ly = (double)y - ybase;
    ci = graded_cell(g.gx, g.nux, lx);
    cj = graded_cell(g.gy, g.nuy, ly);
    a = (lx - g.gx[ci]) / (g.gx[ci + 1] - g.gx[ci]);
    b = (ly - g.gy[cj]) / (g.gy[cj + 1] - g.gy[cj]);
    (void)lowest_triangle(g, ci, cj, [&](int i, int j, double &aa, double &bb) {
      aa = (lx - g.gx[i]) / (g.gx[i + 1] - g.gx[i]);
      bb = (ly - g.gy[j]) / (g.gy[j + 1] - g.gy[j]);
    }, ci, cj, a, b, tri);
    return;
  }
  const double X0 = g.xc + (double)(0 - g.nux / 2) * g.h;
  const double Y0 = ybase + (0.0 - 0.5 * (double)(g.nuy - 1)) * g.h;
  const double s = ((double)x - X0) / g.h, t = ((double)y - Y0) / g.h;
  ci = min(max((int)floor(s), 0), g.nux - 2);
  cj = min(max((int)floor(t), 0), g.nuy - 2);
  a = s - ci;
  b = t - cj;
  (void)lowest_triangle(g, ci, cj, [&](int i, int j, double &aa, double &bb) {
    aa = s - i;
    bb = t - j;
  }, ci, cj, a, b, tri);
}

// Refill classification of grid node (i, j) moved from ybase to ybase1
// (Sec. Refill procedure): 3 = inside a triangle of the old grid (cell ci,
// cj, local a, b), 2 = inside the old lamina, 1 = outside the old grid.
struct RefillCell {
  int kind, ci, cj;
  double a, b;
  int tri;  // triangle of the cell (kind 3)
};

__device__ __forceinline__ RefillCell refill_cell_graded(const GridGeom &g, double ybase, double ybase1, int i,
                                                         int j) {
  // the grid moves in y only: the node keeps its column, and its new height
  // is located among the old rows
  const double xrel = g.gx[i];
  const double Ynew = ybase1 + g.gy[j];
  const double py = Ynew - ybase;
  RefillCell r{0, 0, 0, 0.0, 0.0, -1};
  const int ci0 = min(i, g.nux - 2), cj0 = graded_cell(g.gy, g.nuy, py);
  if (lowest_triangle(g, ci0, cj0, [&](int ci, int cj, double &aa, double &bb) {
        aa = (xrel - g.gx[ci]) / (g.gx[ci + 1] - g.gx[ci]);
        bb = (py - g.gy[cj]) / (g.gy[cj + 1] - g.gy[cj]);
      }, r.ci, r.cj, r.a, r.b, r.tri))
    r.kind = 3;
  else
    r.kind = (g.body && fabs(xrel) < g.half_b && fabs(py) < g.half_T) ? 2 : 1;
  return r;
}

__device__ __forceinline__ RefillCell refill_cell(const GridGeom &g, double ybase, double ybase1, int i, int j) {
  if (g.gx) return refill_cell_graded(g, ybase, ybase1, i, j);
  const double xrel = (double)(i - g.nux / 2) * g.h;
  const double Ynew = ybase1 + ((double)j - 0.5 * (double)(g.nuy - 1)) * g.h;
  const double Y0 = ybase + (0.0 - 0.5 * (double)(g.nuy - 1)) * g.h;
  const double s = (double)i, t = (Ynew - Y0) / g.h;
  RefillCell r{0, 0, 0, 0.0, 0.0, -1};
  const int ci0 = min(max((int)floor(s), 0), g.nux - 2), cj0 = min(max((int)floor(t), 0), g.nuy - 2);
  if (lowest_triangle(g, ci0, cj0, [&](int ci, int cj, double &aa, double &bb) {
        aa = s - ci;
        bb = t - cj;
      }, r.ci, r.cj, r.a, r.b, r.tri))
    r.kind = 3;
  else
    r.kind = (g.body && fabs(xrel) < g.half_b && fabs(Ynew - ybase) < g.half_T) ? 2 : 1;
  return r;
}


// ---- interpolation arithmetic shared by forward and adjoint ---------------------
// Bilinear Lagrange interpolation over the lattice cell around (X, Y) of
// density, velocity and f^neq = f - f^eq of the pre-collision populations at
// t_{k+1} pulled from A (refill type 1 and the grid's interface donors).
template <class T, class R>
__device__ __forceinline__ void lattice_bilinear(const T *__restrict__ A, int nx, int ny, size_t plane, int bc,
                                                 double X, double Y, R &rho, R &ux, R &uy, R fneq[9]) {
  const double fx = floor(X), fy = floor(Y);
  const double a = X - fx, b = Y - fy;
  int x0 = (int)fx, y0 = (int)fy;
  const double w4[4] = {(1.0 - a) * (1.0 - b), a * (1.0 - b), (1.0 - a) * b, a * b};
  rho = ux = uy = R(0);
#pragma unroll
  for (int q = 0; q < 9; ++q) fneq[q] = R(0);
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    int xd = x0 + (d & 1), yd = y0 + (d >> 1);
    xd = xd >= nx ? xd - nx : (xd < 0 ? xd + nx : xd);
    if (bc) yd = yd >= ny ? yd - ny : (yd < 0 ? yd + ny : yd);
    R f[9], e[9], r, vx, vy;
    pull<T, R>(A, nx, ny, plane, bc, xd, yd, f);
    moments<R>(f, r, vx, vy);
    equilibrium<R>(r, vx, vy, e);
    const R w = R(w4[d]);
    rho += w * r;
    ux += w * vx;
    uy += w * vy;
#pragma unroll
    for (int q = 0; q < 9; ++q) fneq[q] += w * (f[q] - e[q]);
  }
}

// One lane's share of an interface node's donors: corner d of the lattice
// cell around (X, Y), weighted (rho, u_x, u_y, f^neq[9]) in acc[12].
template <class T, class R>
__device__ __forceinline__ void donor_corner(const T *__restrict__ A, int nx, int ny, size_t plane, int bc,
                                             double X, double Y, int d, R acc[12]) {
  const double fx = floor(X), fy = floor(Y);
  const double a = X - fx, b = Y - fy;
  const double w = (d & 1 ? a : 1.0 - a) * (d >> 1 ? b : 1.0 - b);
  int xd = (int)fx + (d & 1), yd = (int)fy + (d >> 1);
  xd = xd >= nx ? xd - nx : (xd < 0 ? xd + nx : xd);
  if (bc) yd = yd >= ny ? yd - ny : (yd < 0 ? yd + ny : yd);
  R f[9], e[9], r, vx, vy;
  pull<T, R>(A, nx, ny, plane, bc, xd, yd, f);
  moments<R>(f, r, vx, vy);
  equilibrium<R>(r, vx, vy, e);
  const R wr = R(w);
  acc[0] = wr * r;
  acc[1] = wr * vx;
  acc[2] = wr * vy;
#pragma unroll
  for (int q = 0; q < 9; ++q) acc[3 + q] = wr * (f[q] - e[q]);
}

// Barycentric interpolation of rho, u and f^neq,u of grid state g over a
// triangle (lattice interpolation nodes, Eq.(postcollision2_s)).
template <class R>
__device__ __forceinline__ void grid_barycentric(const R *__restrict__ g, int nnode, const int node[3],
                                                 const double lam[3], R &rho, R &ux, R &uy, R fneq[9]) {
  rho = ux = uy = R(0);
#pragma unroll
  for (int q = 0; q < 9; ++q) fneq[q] = R(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    R f[9], e[9], r, vx, vy;
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q] = g[(size_t)q * nnode + node[a]];
    moments<R>(f, r, vx, vy);
    equilibrium<R>(r, vx, vy, e);
    const R l = R(lam[a]);
    rho += l * r;
    ux += l * vx;
    uy += l * vy;
#pragma unroll
    for (int q = 0; q < 9; ++q) fneq[q] += l * (f[q] - e[q]);
  }
}

// Lattice nodes set from the grid at step k: interpolation nodes (inside the
// fictitious rectangle on its edge) and nodes the rectangle uncovered since
// step k - 1.
__device__ __forceinline__ bool from_grid_target(const StepParams &P, int x, int y) {
  const bool in_k = x >= P.ix0 && x <= P.ix1 && y >= P.iy0 && y <= P.iy1;
  const bool in_p = x >= P.pix0 && x <= P.pix1 && y >= P.piy0 && y <= P.piy1;
  const bool interp = in_k && (x == P.ix0 || x == P.ix1 || y == P.iy0 || y == P.iy1);
  return interp || (!in_k && in_p);
}

}  // namespace dev
}  // namespace mghlbm
