// Internal declarations of the gfx950 HLBM library: device-side data layouts
// shared by the host runtime and the kernels. Nothing here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <string>
#include <vector>

namespace mghlbm {

// The grid is a split-quad mesh, so every finite-volume stencil lies in the
// 3 x 3 node neighbourhood; stencils are stored densely over its nine slots,
// slot = (dj + 1) * 3 + (di + 1); slot 4 is the node itself.
constexpr int NSLOT = 9;
constexpr int SELF_SLOT = 4;

enum NodeType : int { NODE_INTERIOR = 0, NODE_INTERFACE = 1, NODE_WALL = 2 };

// Per-structured-step scalars, computed once on the host in FP64 so the
// discrete decisions (node status, donor cells) use the same bits as any
// other FP64 implementation of the same formulas.
struct StepParams {
  double y;      // lamina offset y(t_k) = A sin(omega k)
  double y1;     // y(t_{k+1})
  double ybase;  // yc + y(t_k): absolute y of the grid centre line at t_k
  double ybase1; // yc + y(t_{k+1})
  int ix0, ix1, iy0, iy1;      // lattice nodes inside the fictitious rectangle at t_k
  int pix0, pix1, piy0, piy1;  // same at t_{k-1} (t_0 for k = 0)
  double beta, beta1;  // bending amplitude of a deforming grid at t_k, t_{k+1} (0: rigid)
};

// One finite-volume stencil shared by every grid node with the same
// neighbourhood geometry and role (Eq.(ulbe) coefficients). The streaming
// matrix factors as S_ik = c_ix Gx_k + c_iy Gy_k, where (Gx, Gy)_k are the
// weights of the control-volume gradient, G_k = -(1/V_P) sum_T (|T|/3)
// grad(phi_k on T); so a stencil is 27 numbers. A slot holds a neighbour
// exactly when its C entry is non-zero (C_ik > 0 for neighbours).
template <class R>
struct GridClass {
  R Gx[NSLOT];      // x weights of the streaming matrix
  R Gy[NSLOT];      // y weights of the streaming matrix
  R C[NSLOT];       // collision matrix C_ik
  int type;         // NodeType
  int zero_diag;    // bit 0: slots 2 and 6 (the (+1,-1) and (-1,+1)
                    // neighbours) carry zero weights; bit 1: slots 0 and 8
};

// slots a split-quad node lacks: the two diagonal neighbours across the
// diagonals its cells are not split along
constexpr int kZeroDiag26 = 1, kZeroDiag08 = 2;

struct WallEdge {
  int a, b;         // node indices
  double nx, ny;    // unit normal pointing out of the body
  double len;
};

// Host-side body-fitted grid (built independently of any other
// implementation from the definition of the lamina grid).
struct HostGrid {
  int nux = 0, nuy = 0;
  double h = 1.0, b = 0.0, T = 0.0;
  bool body = false;
  int nnode = 0, ntri = 0;
  std::vector<int> type;                 // NodeType per node
  std::vector<int> cls;                  // class id per node
  std::vector<GridClass<double>> classes;
  std::vector<int> iface;                // interface (outer ring) node ids
  std::vector<WallEdge> wall;            // body polygon edges
  // unstructured grid (build_mesh; no classes then)
  bool mesh = false;
  std::vector<double> x, y;              // node coordinates, local frame
  std::vector<int> tri;                  // [ntri][3] counter-clockwise
  std::vector<double> txy;               // [ntri][3][2] vertex coordinates
  std::vector<int> row, col;             // stencil of node p: col[row[p] .. row[p+1]), the node first
  std::vector<double> C, Gx, Gy;         // its weights, per entry
  // triangles around node p: tlist[trow[p] .. trow[p+1]) in increasing
  // order, with the stencil slot (entry - row[p]) of each of their three
  // vertices in bits 10a .. 10a+9 of tslot
  std::vector<int> trow, tlist, tslot;
  std::vector<int> wall_o;               // third vertex of each wall edge's triangle
  double ex0 = 0, ex1 = 0, ey0 = 0, ey1 = 0;  // bounding box of the nodes
  // point location: unit buckets over the bounding box, each listing (in
  // increasing order) the triangles whose box, grown by one bucket, meets it
  double bx0 = 0, by0 = 0;
  int bnx = 0, bny = 0;
  std::vector<int> bstart, blist;
};

// bucket size of the unstructured grid's point location (lattice units)
constexpr double kBucket = 1.0;

// Device view of an unstructured grid's point-location data.
struct MeshGeom {
  const int *tri;      // [ntri][3]
  const double *txy;   // [ntri][3][2]
  const int *bstart;   // [bnx * bny + 1]
  const int *blist;
  double bx0, by0;
  int bnx, bny;
};

// Builds the grid, its median-dual finite-volume matrices and stencil
// classes. Returns false with a message on invalid geometry.
// gx, gy (optional): local x of each column and y of each row of a graded grid.
bool build_grid(int nux, int nuy, double h, double b, bool body, HostGrid *g, std::string *err,
                const double *gx = nullptr, const double *gy = nullptr);

// An unstructured grid: nodes at local xy [nnode][2] with types [nnode]
// (NodeType), counter-clockwise triangles tri [ntri][3]; the lamina is
// |x| < b/2, |y| < T/2 (body). Builds the per-node stencils of the same
// median-dual matrices, the wall edges and the point-location buckets.
// False with a message when the mesh is not a valid grid of the region:
// indices or types out of range, a triangle without positive area, an
// edge shared by more than two triangles, a boundary edge whose ends are
// not both interface nodes or both wall nodes, interface nodes off the
// bounding box, a bounding box not symmetric about y = 0.
bool build_mesh(int nnode, const double *xy, const int *type, int ntri, const int *tri, double b, double T,
                bool body, HostGrid *g, std::string *err);

}  // namespace mghlbm
