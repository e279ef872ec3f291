// Launch interface of the gfx950 HLBM kernels (internal to the library).
#pragma once

#include "hlbm_internal.h"

namespace mghlbm {

// Two-way coupled motion of the lamina: M y'' + C y' + K y = F_y per unit
// depth, advanced by the force kernel, which also fills the next step's
// scalars (the rectangle rows as the host computes them: ceil((yc + y) + c0
// + margin), floor((yc + y) + c1 - margin)) and wall velocities.
struct MotionCtx {
  int on;
  double M, K, C, y_max;
  double yc, c0, c1, margin;
  double *state;  // [max_steps + 1][2]: (y, v) at t_k
  int64_t cap;    // max_steps
};

// Everything a kernel of one case needs, by value. Pointers are device
// pointers; the lattice pointers are swapped by the host between steps.
template <class T, class R>
struct CaseView {
  // lattice
  const T *A;      // post-collision populations at t_k, [9][ny][nx]
  T *B;            // post-collision populations at t_{k+1}
  int nx, ny;
  size_t plane;    // elements from one population plane to the next (>= nx * ny)
  int bc;          // HLBM_BC_*: 0 periodic x + y walls, 1 periodic, 2 x walls + y outflow,
                   // 3 outermost ring written from a coarser level (not updated here)
  // nodes strictly inside (sx0, sx1) x (sy0, sy1) are neither read nor
  // written by the stream-collide (a finer level covers them); empty: 0
  int sx0, sx1, sy0, sy1;
  // window of nodes a single-step stream-collide updates: [wx0, wx0 + ww)
  // x [wy0, wy0 + wh) (the whole lattice unless a two-step launch covers
  // the rest)
  int wx0, wy0, ww, wh;
  // two steps per launch: C receives the state at t_{k+2} outside the band
  // [bx0, bx1] x [by0, by1] (inclusive; empty when bx0 > bx1), where the
  // grid coupling needs every step; B receives t_{k+1} on the band and one
  // node around it
  T *C;
  int bx0, bx1, by0, by1;
  MotionCtx mot;
  R inv_tau;       // 1 / tau_s
  R g_post;        // 2 (tau_s - 1) / (2 tau_s - 1), Eq.(postcollision2_s)
  R k_neq;         // 1 - 1/(2 tau_s), Eq.(continuity_stresses)
  int has_grid;
  // grid
  int nux, nuy, nnode, n_iface, n_wall_edges, n_sub;
  double h, xc, yc, half_b, half_T;
  int body;
  const double *gx, *gy;  // graded grid: local x of each column, y of each row (null: uniform)
  // per grid node: 16 class + 4 zero_diag + type of its stencil class
  // (-1: no class), so a kernel learns a node's type and stencil in one load
  const int *ncode;
  const GridClass<R> *tab;
  const int *iface;
  const WallEdge *wall;
  // unstructured grid (mesh != 0; the split-quad fields above unused):
  // stencil of node p at entries m_row[p] .. m_row[p+1]-1 (node ids m_col,
  // weights m_C, m_Gx, m_Gy), node coordinates and types, triangles and
  // the point-location buckets
  int mesh;
  const int *m_row, *m_col;
  const R *m_C, *m_Gx, *m_Gy;
  const double *m_x, *m_y;
  const int *m_type;
  MeshGeom mg;
  // a bending unstructured grid (deform != 0): node p's local y at step k
  // is m_yref[p] + m_prof[p] beta_k; a wall node's bending velocity is
  // uwb[k n_sub + m] m_sx[p] on top of uw
  int deform;
  const double *m_yref, *m_prof;
  const R *m_sx, *uwb;
  R *star_f;       // [9][nnode] structured-derived f* at interface nodes
  R *star_n;       // [9][nnode] structured-derived f^neq* at interface nodes
  R dt_u, dt_over_tau_u;
  const R *uw;     // wall velocity table [max_steps][n_sub]
  const StepParams *params;  // [max_steps + 1]
  int64_t *dk;     // device step counter
  const int64_t *dkl;  // the step the two-step lattice launch reads (dk, or a
                       // copy taken before a grid path that runs beside it)
  double *hist;    // [max_steps][2]
  int *flag;       // non-finite force seen
  unsigned long long *counts;  // refill type 1 and type 2 counters
  // lattice rows and columns the interpolation kernel must cover
  int k2_x0, k2_w, k2_h;
  // case-batched kernels pick their buffers from the step counter:
  // lattice lat[k & 1] -> lat[(k + 1) & 1], grid buffers by flip parity
  T *lat[2];
  R *grid[2];
  int64_t max_steps;  // a batched case stops here
};

// What the geometry update of a bending unstructured grid writes and reads
// (device pointers): the configuration of step *dk (node p at local x[p],
// yref[p] + prof[p] params[*dk].beta) gives the stencil weights C, Gx, Gy
// (entries row[p] .. row[p+1]-1), the triangles' vertex coordinates txy and
// the wall edges' normals and lengths (wall_o: the third vertex of each
// wall edge's triangle).
template <class R>
struct MeshDeformView {
  int nnode, ntri, nwall;
  const double *x, *yref, *prof;
  const int *tri, *row, *trow, *tlist, *tslot, *wall_o;
  R *C, *Gx, *Gy;
  double *txy;
  WallEdge *wall;
  const StepParams *params;
  const int64_t *dk;
};

// Population-plane stride of lattice buffers: nx * ny rounded up to 256
// nodes plus 2112. Planes a power of two apart put the nine streams of the
// stream-collide on the same HBM channels at once; the offset spreads them.
inline size_t lattice_plane(int nx, int ny) {
  return (((size_t)nx * ny + 255) / 256) * 256 + 2112;
}

enum class BatchKernel { StreamCollide, LatticeFromGrid, InterfaceDonors, GridSubsteps, Refill, Force };

// one phase of a persistent batched step: block function `which`
// (BatchKernel), work items first .. first+n-1, first sub-step m0
struct BatchPhase {
  int which, first, n, m0;
};

// grid sub-steps advanced per launch (temporal blocking depth)
constexpr int kSubstepBlock = 4;

// default launch shape of the lattice stream-collide: workgroup width and
// rows per lane
constexpr int kLatticeThreads = 128, kLatticeRows = 2;
// tile of the two-step stream-collide
constexpr int kTwoStepTX = 64, kTwoStepTY = 8;

// Variants of the grid sub-step kernel (tile of grid nodes per workgroup,
// workgroup size):
//   0: 16 x 16, 576 threads   1: 32 x 8, 640 threads
//   2: 64 x 4, 896 threads    3: 16 x 8, 384 threads
//   4: 8 x 8, 64 threads      5: 16 x 8, 128 threads
//   6: 16 x 16, 256 threads   7: 8 x 4, 64 threads
// (4-7: several nodes per lane, more workgroups per CU), all advancing up to
// kSubstepBlock sub-steps per launch; single cases also take
//   8: 32 x 8, 256 threads, one sub-step per launch
//   9: 16 x 16, 256 threads, one sub-step per launch
//  10: 32 x 8, 384 threads, two sub-steps per launch
// (large grids, where the halo updates of deeper blocking cost more than
// the loads they save)
constexpr int kSubstepVariants = 8;         // case-batched kernels
constexpr int kSubstepVariantsSingle = 11;  // single-case kernels
// sub-steps a launch of `variant` advances at most (callers step by it)
int substep_block(int variant);
template <class R>
constexpr int default_substep_variant() {
  return sizeof(R) == 8 ? 1 : 3;  // fastest at the 512 x 128 grid (hlbm_tune measures)
}
// tile shape of a sub-step variant (work lists of the batched kernel)
void substep_tile(int variant, int *tx, int *ty);

template <class T, class R>
struct Kernels {
  static hipError_t prepare();  // one-time launch attributes (dynamic LDS of the sub-step)
  static void fill_rest(T *lat, size_t plane, R *grid, int nnode, hipStream_t s);  // whole planes
  // start/stop (optional): events recorded at the kernel's own start and end
  // threads x rows: workgroup width and lattice rows per lane (1, 2 or 4);
  // <= 0 takes kLatticeThreads / kLatticeRows; order 1: each XCD takes a
  // contiguous band of rows; donors: the same launch also computes the
  // grid's interface donors from v.A (as interface_donors), in workgroups of
  // its own
  static void stream_collide(const CaseView<T, R> &v, hipStream_t s, hipEvent_t start = nullptr,
                             hipEvent_t stop = nullptr, int threads = 0, int rows = 0, int order = 0,
                             bool donors = false);
  // two steps t_k -> t_{k+2} in one launch (tile of kTwoStepTX x kTwoStepTY
  // nodes, the first step on the tile and a one-node ring kept in LDS);
  // needs nx >= kTwoStepTX + 2 and ny >= kTwoStepTY + 2; order 1: the
  // tiles are dealt to the XCDs in contiguous runs of rows, each XCD
  // starting at a different offset (0: in turn, row by row); donors: as
  // for stream_collide
  static void stream_collide2(const CaseView<T, R> &v, hipStream_t s, hipEvent_t start = nullptr,
                              hipEvent_t stop = nullptr, int order = 0, bool donors = false);
  static void lattice_from_grid(const CaseView<T, R> &v, const R *grid, hipStream_t s);
  static void interface_donors(const CaseView<T, R> &v, hipStream_t s);
  // one sub-step m of an unstructured grid (Eq.(ulbe), Eq.(postcollision2_u)),
  // one node per lane; optional events at the kernel's own start and end
  static void mesh_substep(const CaseView<T, R> &v, const R *f, R *fout, int m, hipStream_t s,
                           hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
  // sub-steps m0 .. m0+count-1 (count <= kSubstepBlock) in one launch; with
  // a tape, the grid after sub-step m (m0 < m < m0+count) is also stored at
  // tape + m * 9 * nnode, and the moments (rho, u_x, u_y) of every wall node
  // before its velocity is imposed in sub-step m at wtape + (3 m + c) nwall
  // + widx[node]
  // start, stop (optional): events taken at the launch's own start and end
  static void grid_substeps(const CaseView<T, R> &v, const R *f, R *fout, int m0, int count, hipStream_t s,
                            R *tape = nullptr, R *wtape = nullptr, const int *widx = nullptr, int nwall = 0,
                            int variant = -1, hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
  template <int V>
  static void grid_substeps_v(const CaseView<T, R> &v, const R *f, R *fout, int m0, int count, hipStream_t s,
                              R *tape, R *wtape, const int *widx, int nwall, hipEvent_t start, hipEvent_t stop);
  static void refill(const CaseView<T, R> &v, const R *fold, R *fnew, hipStream_t s);
  // geometry of a bending unstructured grid at the current step
  static void mesh_deform(const MeshDeformView<R> &g, hipStream_t s);
  // *to = *from (one lane): a copy of the step counter
  static void copy_step(const int64_t *from, int64_t *to, hipStream_t s);
  // refill and force (prescribed motion) in one launch, then the step
  // counter advances; done: a device counter that starts at 0 and is left at 0
  static void refill_force(const CaseView<T, R> &v, const R *fold, R *fnew, unsigned *done, hipStream_t s);
  // advance = 0: leave the step counter (a coupled-motion step then runs the
  // refill and advance_step after it)
  static void force(const CaseView<T, R> &v, const R *f, hipStream_t s, int advance = 1);
  static void advance_step(const CaseView<T, R> &v, hipStream_t s);
  // between a lattice buffer (plane stride) and a packed [9][nodes] FP64 array
  static void lattice_to_f64(const T *src, double *dst, size_t plane, size_t nodes, hipStream_t s);
  // n consecutive values of population plane q of a lattice buffer (src
  // points at the first), or of a grid array, as FP64 into dst
  static void lattice_stage_f64(const T *src, double *dst, size_t n, int q, hipStream_t s);
  static void grid_stage_f64(const R *src, double *dst, size_t n, hipStream_t s);
  // one launch of a case-batched step over a work list of int4 items
  // (case, block x, block y, 0); GridSubsteps: (case, tile) for sub-steps
  // m0 .. m0+3 of every listed case; threads: stream-collide workgroup size
  // (<= 256), or for GridSubsteps the sub-step variant (-1: default)
  static void batched(BatchKernel which, const CaseView<T, R> *views, const int4 *items, int nitems, int m0,
                      int threads, hipStream_t s, int rows = 1);
  static void lattice_from_f64(const double *src, T *dst, size_t plane, size_t nodes, hipStream_t s);
  // `steps` steps of the running cases in one cooperative launch of at most
  // max_groups workgroups of the sub-step variant's width (variants 4-7),
  // walking the phases prog[0 .. nphase-1] of a step with a grid barrier
  // after each; the work items are built for that width and one lattice row
  // per lane
  static hipError_t batched_persistent(const CaseView<T, R> *views, const int4 *items, const BatchPhase *prog,
                                       int nphase, int steps, int variant, int max_groups, hipStream_t s);
  // workgroup width of the persistent kernel of a sub-step variant (0: none)
  static int persistent_threads(int variant);
};

// Exchange between structured refinement levels. A box (x0, y0, x1, y1) of
// a coarse level is covered by the next finer level; its perimeter nodes are
// numbered p = 0 .. 2 (W + H) - 1 (W = x1 - x0, H = y1 - y0): bottom row
// x0..x1, top row x0..x1, left column y0+1..y1-1, right column y0+1..y1-1.
struct LevelBox {
  int x0, y0, x1, y1;
  int W() const { return x1 - x0; }
  int H() const { return y1 - y0; }
  int perimeter() const { return 2 * (W() + H()); }
};

template <class T, class R>
struct LevelKernels {
  // m [12][nper]: pre-collision (rho, u_x, u_y, f^neq) on the box perimeter,
  // pulled from post-collision buffer P of the coarse level
  static void box_moments(const T *P, int nx, int ny, size_t plane, int bc, LevelBox box, R *m, hipStream_t s);
  // ring of the finer level (nxf x nyf, buffer F): moments m0 at t and m1 at
  // t + 1 weighted (1 - tw1, tw1), f = f^eq + kf f^neq
  static void prolong(const R *m0, const R *m1, LevelBox box, double tw1, double kf, T *F, int nxf, int nyf,
                      size_t planef, hipStream_t s);
  // coarse nodes one inside the box (buffer Cb) from the finer level's
  // pre-collision state pulled from its post-collision buffer Fprev:
  // f = f^eq + kc f^neq
  static void restrict_level(const T *Fprev, int nxf, int nyf, size_t planef, LevelBox box, double kc, T *Cb,
                             int nx, size_t plane, hipStream_t s);
};

extern template struct Kernels<double, double>;
extern template struct Kernels<float, float>;
extern template struct Kernels<__half, float>;
extern template struct LevelKernels<double, double>;
extern template struct LevelKernels<float, float>;
extern template struct LevelKernels<__half, float>;

}  // namespace mghlbm
