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
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <utility>

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

// Unstructured grid. Per node, the stencil holds the vertices of every
// triangle around it (the node first, then by increasing id); the same
// median-dual expressions as above, summed over those triangles:
//   Gx_k = -(1/V_P) sum_T (|T|/3) d(phi_k)/dx,  Gy_k likewise,
//   C_k  =  (1/V_P) sum_T |T| (11/54 for k = P, 7/108 otherwise),
//   V_P  =  sum_T |T|/3.
bool build_mesh(int nnode, const double *xy, const int *type, int ntri, const int *tri, double b, double T,
                bool body, HostGrid *g, std::string *err) {
  if (nnode < 3 || ntri < 1 || !xy || !type || !tri) {
    *err = "mesh needs at least 3 nodes and 1 triangle";
    return false;
  }
  g->mesh = true;
  g->nux = g->nuy = 0;
  g->h = 1.0;
  g->b = body ? b : 0.0;
  g->T = body ? T : 0.0;
  g->body = body;
  g->nnode = nnode;
  g->ntri = ntri;
  g->x.resize(nnode);
  g->y.resize(nnode);
  g->type.resize(nnode);
  g->cls.clear();
  g->classes.clear();
  int nwall = 0, nface = 0;
  for (int p = 0; p < nnode; ++p) {
    g->x[p] = xy[2 * p];
    g->y[p] = xy[2 * p + 1];
    const int t = type[p];
    if (t != NODE_INTERIOR && t != NODE_INTERFACE && t != NODE_WALL) {
      *err = "mesh node type out of range";
      return false;
    }
    g->type[p] = t;
    nwall += t == NODE_WALL;
    nface += t == NODE_INTERFACE;
  }
  if (nface == 0 || (body && nwall == 0) || (!body && nwall > 0)) {
    *err = body ? "mesh needs interface nodes and wall nodes" : "mesh without a body has wall nodes or no interface";
    return false;
  }
  g->ex0 = *std::min_element(g->x.begin(), g->x.end());
  g->ex1 = *std::max_element(g->x.begin(), g->x.end());
  g->ey0 = *std::min_element(g->y.begin(), g->y.end());
  g->ey1 = *std::max_element(g->y.begin(), g->y.end());
  if (!(g->ey1 > 0.0 && std::fabs(g->ey0 + g->ey1) <= 1e-12 * g->ey1)) {
    *err = "mesh bounding box not symmetric about y = 0";
    return false;
  }
  g->tri.assign(tri, tri + 3 * (size_t)ntri);
  g->txy.resize(6 * (size_t)ntri);
  std::vector<std::vector<int>> around(nnode);  // triangles around each node
  for (int t = 0; t < ntri; ++t) {
    for (int a = 0; a < 3; ++a) {
      const int id = tri[3 * t + a];
      if (id < 0 || id >= nnode) {
        *err = "mesh triangle index out of range";
        return false;
      }
      g->txy[6 * t + 2 * a] = g->x[id];
      g->txy[6 * t + 2 * a + 1] = g->y[id];
      around[id].push_back(t);
    }
    const double *q = &g->txy[6 * t];
    if (!((q[2] - q[0]) * (q[5] - q[1]) - (q[4] - q[0]) * (q[3] - q[1]) > 0.0)) {
      *err = "mesh triangle not counter-clockwise with positive area";
      return false;
    }
  }
  // edges: interior ones shared by two triangles, boundary ones by one
  std::map<std::pair<int, int>, std::vector<int>> edges;  // (lo, hi) -> (triangle, third vertex) pairs
  for (int t = 0; t < ntri; ++t)
    for (int e = 0; e < 3; ++e) {
      const int a = tri[3 * t + e], c = tri[3 * t + (e + 1) % 3], o = tri[3 * t + (e + 2) % 3];
      auto &v = edges[{std::min(a, c), std::max(a, c)}];
      v.push_back(t);
      v.push_back(o);
    }
  g->wall.clear();
  g->wall_o.clear();
  const double tol = 1e-12 * std::max({g->ex1 - g->ex0, g->ey1 - g->ey0, 1.0});
  auto on_box = [&](int p) {
    return std::fabs(g->x[p] - g->ex0) <= tol || std::fabs(g->x[p] - g->ex1) <= tol ||
           std::fabs(g->y[p] - g->ey0) <= tol || std::fabs(g->y[p] - g->ey1) <= tol;
  };
  for (const auto &kv : edges) {
    const int a = kv.first.first, c = kv.first.second;
    if (kv.second.size() > 4) {
      *err = "mesh edge shared by more than two triangles";
      return false;
    }
    if (kv.second.size() == 4) continue;
    if (g->type[a] != g->type[c] || g->type[a] == NODE_INTERIOR) {
      *err = "mesh boundary edge whose ends are not both interface or both wall nodes";
      return false;
    }
    if (g->type[a] == NODE_WALL) {
      // unit normal out of the body: toward the triangle's third vertex
      const int o = kv.second[1];
      const double ex = g->x[c] - g->x[a], ey = g->y[c] - g->y[a];
      const double len = std::sqrt(ex * ex + ey * ey);
      double nx = -ey / len, ny = ex / len;
      if (nx * (g->x[o] - g->x[a]) + ny * (g->y[o] - g->y[a]) < 0.0) {
        nx = -nx;
        ny = -ny;
      }
      g->wall.push_back({a, c, nx, ny, len});
      g->wall_o.push_back(o);
    }
  }
  g->iface.clear();
  for (int p = 0; p < nnode; ++p) {
    if (around[p].empty()) {
      *err = "mesh node in no triangle";
      return false;
    }
    if (g->type[p] == NODE_INTERFACE) {
      if (!on_box(p)) {
        *err = "mesh interface node off the bounding box";
        return false;
      }
      g->iface.push_back(p);
    }
  }
  // stencils
  g->row.assign(nnode + 1, 0);
  g->col.clear();
  g->C.clear();
  g->Gx.clear();
  g->Gy.clear();
  g->trow.assign(nnode + 1, 0);
  g->tlist.clear();
  g->tslot.clear();
  for (int p = 0; p < nnode; ++p) {
    std::vector<int> nb;
    for (int t : around[p])
      for (int a = 0; a < 3; ++a)
        if (tri[3 * t + a] != p) nb.push_back(tri[3 * t + a]);
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    nb.insert(nb.begin(), p);
    std::vector<double> C(nb.size(), 0.0), Gx(nb.size(), 0.0), Gy(nb.size(), 0.0);
    double V = 0.0;
    for (int t : around[p]) {
      const double *q = &g->txy[6 * t];
      const double area = 0.5 * ((q[2] - q[0]) * (q[5] - q[1]) - (q[4] - q[0]) * (q[3] - q[1]));
      V += area / 3.0;
      for (int a = 0; a < 3; ++a) {
        const int ab = (a + 1) % 3, ac = (a + 2) % 3;
        const double dphx = -(q[2 * ac + 1] - q[2 * ab + 1]) / (2.0 * area);
        const double dphy = (q[2 * ac] - q[2 * ab]) / (2.0 * area);
        const int k = (int)(std::lower_bound(nb.begin() + 1, nb.end(), tri[3 * t + a]) - nb.begin());
        const int s = tri[3 * t + a] == p ? 0 : k;
        Gx[s] -= (area / 3.0) * dphx;
        Gy[s] -= (area / 3.0) * dphy;
        C[s] += area * (tri[3 * t + a] == p ? 11.0 / 54.0 : 7.0 / 108.0);
      }
    }
    if (nb.size() > 1024) {
      *err = "mesh node with more than 1023 neighbours";
      return false;
    }
    for (int t : around[p]) {
      int packed = 0;
      for (int a = 0; a < 3; ++a) {
        const int q = tri[3 * t + a];
        const int s = q == p ? 0 : (int)(std::lower_bound(nb.begin() + 1, nb.end(), q) - nb.begin());
        packed |= s << (10 * a);
      }
      g->tlist.push_back(t);
      g->tslot.push_back(packed);
    }
    g->trow[p + 1] = (int)g->tlist.size();
    for (size_t s = 0; s < nb.size(); ++s) {
      g->col.push_back(nb[s]);
      g->C.push_back(C[s] / V);
      g->Gx.push_back(Gx[s] / V);
      g->Gy.push_back(Gy[s] / V);
    }
    g->row[p + 1] = (int)g->col.size();
  }
  // point-location buckets
  g->bx0 = g->ex0;
  g->by0 = g->ey0;
  g->bnx = (int)std::floor((g->ex1 - g->ex0) / kBucket) + 1;
  g->bny = (int)std::floor((g->ey1 - g->ey0) / kBucket) + 1;
  const size_t nb = (size_t)g->bnx * g->bny;
  std::vector<std::vector<int>> lists(nb);
  for (int t = 0; t < ntri; ++t) {
    const double *q = &g->txy[6 * t];
    const double x0 = std::min({q[0], q[2], q[4]}), x1 = std::max({q[0], q[2], q[4]});
    const double y0 = std::min({q[1], q[3], q[5]}), y1 = std::max({q[1], q[3], q[5]});
    const int i0 = std::max(0, (int)std::floor((x0 - g->bx0) / kBucket) - 1);
    const int i1 = std::min(g->bnx - 1, (int)std::floor((x1 - g->bx0) / kBucket) + 1);
    const int j0 = std::max(0, (int)std::floor((y0 - g->by0) / kBucket) - 1);
    const int j1 = std::min(g->bny - 1, (int)std::floor((y1 - g->by0) / kBucket) + 1);
    for (int j = j0; j <= j1; ++j)
      for (int i = i0; i <= i1; ++i) lists[(size_t)j * g->bnx + i].push_back(t);
  }
  g->bstart.assign(nb + 1, 0);
  g->blist.clear();
  for (size_t i = 0; i < nb; ++i) {
    g->blist.insert(g->blist.end(), lists[i].begin(), lists[i].end());
    g->bstart[i + 1] = (int)g->blist.size();
  }
  return true;
}

}  // namespace mghlbm
