// Body-fitted grid of the lamina and its finite-volume matrices (host side).
//
// Grid (Sec. HLBM: unstructured triangular mesh around the body): nux*nuy
// nodes with spacing h, node (i, j) at local x = (i - nux/2) h,
// y = (j - (nuy-1)/2) h, or graded: column i at x = gx[i], row j at
// y = gy[j] (the lamina thickness is then gy[nuy/2] - gy[nuy/2-1]). Each quad cell is cut into two triangles along a
// diagonal that is mirrored about the centre line x = 0 (rising diagonal for
// cells left of it), so the grid is left-right symmetric. The lamina of width
// b and thickness h fills the cells between rows nuy/2-1 and nuy/2 with
// |x| <= b/2, which are not meshed.
//
// Finite-volume matrices of Eq.(ulbe) (cited, not printed, in the paper):
// median-dual control volumes (each triangle gives a third of its area to
// each vertex) with f linear on every triangle. For such f the outflow of
// population i through the closed control-volume boundary equals, by the
// divergence theorem, the integral of c_i . grad f over the volume, so
//     S_ik = -(1/V_P) sum_{T contains P} (|T|/3) c_i . grad(phi_k on T)
//          = c_ix Gx_k + c_iy Gy_k,
// and the consistent collision matrix is
//     C_ik = (1/V_P) sum_{T} integral over (CV_P in T) of phi_k,
// which is 11/54 |T| for k = P and 7/108 |T| for the other two vertices.
#include <cmath>
#include <cstring>
#include <map>

#include "hlbm_internal.h"

namespace mghlbm {
namespace {

struct Tri {
  int v[3];         // corner ids within the cell: 0=(0,0) 1=(1,0) 2=(0,1) 3=(1,1)
};

// the two triangles of a cell, counter-clockwise
void cell_triangles(bool rising, Tri out[2]) {
  if (rising) {
    out[0] = {{0, 1, 3}};
    out[1] = {{0, 3, 2}};
  } else {
    out[0] = {{0, 1, 2}};
    out[1] = {{1, 3, 2}};
  }
}

}  // namespace

bool build_grid(int nux, int nuy, double h, double b, bool body, HostGrid *g, std::string *err, const double *gx,
                const double *gy) {
  if (nux < 4 || nuy < 4 || (nuy % 2) != 0 || !(h > 0.0) || (body && !(b > 0.0))) {
    *err = "grid needs nux >= 4, even nuy >= 4, h > 0 and b > 0 with a body";
    return false;
  }
  const bool graded = gx != nullptr;
  if (graded) {
    for (int i = 0; i + 1 < nux; ++i)
      if (!(gx[i + 1] > gx[i])) {
        *err = "graded grid columns must increase";
        return false;
      }
    for (int j = 0; j + 1 < nuy; ++j)
      if (!(gy[j + 1] > gy[j])) {
        *err = "graded grid rows must increase";
        return false;
      }
  }
  // cell widths and node positions: uniform spacing h, or the given columns and rows
  const double T = graded ? gy[nuy / 2] - gy[nuy / 2 - 1] : h;
  g->nux = nux;
  g->nuy = nuy;
  g->h = h;
  g->b = body ? b : 0.0;
  g->T = body ? T : 0.0;
  g->body = body;
  const int N = nux * nuy;
  g->nnode = N;
  auto xl = [&](int i) { return graded ? gx[i] : (double)(i - nux / 2) * h; };
  auto wxc = [&](int ci) { return graded ? gx[ci + 1] - gx[ci] : h; };
  auto wyc = [&](int cj) { return graded ? gy[cj + 1] - gy[cj] : h; };
  const double half = 0.5 * b + 1e-9 * T;
  const int slot_row = nuy / 2 - 1;
  auto body_cell = [&](int ci, int cj) {
    return body && cj == slot_row && xl(ci) >= -half && xl(ci + 1) <= half;
  };
  auto rising = [&](int ci) { return 2 * ci + 1 < nux; };  // cell centre left of x = 0

  g->type.assign(N, NODE_INTERIOR);
  for (int j = 0; j < nuy; ++j)
    for (int i = 0; i < nux; ++i) {
      int t = NODE_INTERIOR;
      if (body && (j == slot_row || j == slot_row + 1) && std::fabs(xl(i)) <= half) t = NODE_WALL;
      else if (i == 0 || j == 0 || i == nux - 1 || j == nuy - 1) t = NODE_INTERFACE;
      g->type[j * nux + i] = t;
    }
  int ntri = 0;
  for (int cj = 0; cj < nuy - 1; ++cj)
    for (int ci = 0; ci < nux - 1; ++ci)
      if (!body_cell(ci, cj)) ntri += 2;
  g->ntri = ntri;

  // per node: the (up to four) cells around it, visited in a fixed local
  // order so nodes with the same neighbourhood get bit-identical sums
  std::map<std::vector<uint64_t>, int> class_of;
  g->cls.assign(N, 0);
  g->classes.clear();
  for (int j = 0; j < nuy; ++j)
    for (int i = 0; i < nux; ++i) {
      const int p = j * nux + i;
      double V = 0.0;
      double Gx[NSLOT] = {}, Gy[NSLOT] = {}, C[NSLOT] = {};
      for (int dj = -1; dj <= 0; ++dj)
        for (int di = -1; di <= 0; ++di) {
          const int ci = i + di, cj = j + dj;
          if (ci < 0 || cj < 0 || ci >= nux - 1 || cj >= nuy - 1 || body_cell(ci, cj)) continue;
          const int me = (-di) + 2 * (-dj);  // corner id of p in this cell
          const double wx = wxc(ci), wy = wyc(cj);
          const double Xc[4] = {0.0, wx, 0.0, wx}, Yc[4] = {0.0, 0.0, wy, wy};
          Tri tris[2];
          cell_triangles(rising(ci), tris);
          for (const Tri &t : tris) {
            int a = -1;
            for (int s = 0; s < 3; ++s)
              if (t.v[s] == me) a = s;
            if (a < 0) continue;
            const double x0 = Xc[t.v[0]], y0 = Yc[t.v[0]], x1 = Xc[t.v[1]], y1 = Yc[t.v[1]];
            const double x2 = Xc[t.v[2]], y2 = Yc[t.v[2]];
            const double area = 0.5 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0));
            const double px[3] = {x0, x1, x2}, py[3] = {y0, y1, y2};
            V += area / 3.0;
            for (int q = 0; q < 3; ++q) {
              const int qb = (q + 1) % 3, qc = (q + 2) % 3;
              const double dphx = -(py[qc] - py[qb]) / (2.0 * area);
              const double dphy = (px[qc] - px[qb]) / (2.0 * area);
              const int cq = t.v[q];
              const int sdi = (cq & 1) - (me & 1), sdj = (cq >> 1) - (me >> 1);
              const int s = (sdj + 1) * 3 + (sdi + 1);
              Gx[s] -= (area / 3.0) * dphx;
              Gy[s] -= (area / 3.0) * dphy;
              C[s] += area * (q == a ? 11.0 / 54.0 : 7.0 / 108.0);
            }
          }
        }
      if (!(V > 0.0)) {
        *err = "grid node without control volume";
        return false;
      }
      GridClass<double> gc;
      std::memset(&gc, 0, sizeof(gc));
      gc.type = g->type[p];
      for (int s = 0; s < NSLOT; ++s) {
        gc.C[s] = C[s] / V;
        gc.Gx[s] = Gx[s] / V;
        gc.Gy[s] = Gy[s] / V;
      }
      std::vector<uint64_t> key(sizeof(gc) / 8 + 1, 0);
      std::memcpy(key.data(), &gc, sizeof(gc));
      auto it = class_of.find(key);
      if (it == class_of.end()) {
        it = class_of.emplace(key, (int)g->classes.size()).first;
        g->classes.push_back(gc);
      }
      g->cls[p] = it->second;
    }

  g->iface.clear();
  for (int p = 0; p < N; ++p)
    if (g->type[p] == NODE_INTERFACE) g->iface.push_back(p);

  // body polygon: top and bottom faces, then the two end faces
  g->wall.clear();
  if (body) {
    int i0 = -1, i1 = -1;
    for (int i = 0; i < nux; ++i)
      if (std::fabs(xl(i)) <= half) {
        if (i0 < 0) i0 = i;
        i1 = i;
      }
    const int top = slot_row + 1, bot = slot_row;
    for (int i = i0; i < i1; ++i) {
      g->wall.push_back({top * nux + i, top * nux + i + 1, 0.0, 1.0, wxc(i)});
      g->wall.push_back({bot * nux + i, bot * nux + i + 1, 0.0, -1.0, wxc(i)});
    }
    g->wall.push_back({bot * nux + i0, top * nux + i0, -1.0, 0.0, T});
    g->wall.push_back({bot * nux + i1, top * nux + i1, 1.0, 0.0, T});
  }
  return true;
}

}  // namespace mghlbm
