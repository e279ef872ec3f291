// gfx950 kernels of the moving-grid hybrid lattice Boltzmann step.
//
// Storage: structure of arrays, one plane per D2Q9 population, [9][ny][nx]
// for the lattice and [9][nnode] for the body-fitted grid. T is the storage
// type of the lattice and R the arithmetic type (FP64/FP64, FP32/FP32,
// FP16 holding f_i - w_i / FP32). The grid is kept in R.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <type_traits>
#include <cmath>

#include "device_common.h"
#include "kernels.h"

namespace mghlbm {
namespace {

using namespace dev;

// Each kernel body is a per-workgroup device function; a single-case kernel
// takes its block coordinates from the grid, a case-batched kernel takes
// (case, block) from a work list and picks the case's buffers from its step
// counter (lattice buffers alternate every step; the grid buffers flip once
// per sub-step launch and once in the refill).
template <class T, class R>
__device__ __forceinline__ bool batched_case(const CaseView<T, R> &v, int64_t &k) {
  k = *v.dk;
  return k < v.max_steps && *v.flag == 0;
}
template <class T, class R>
__device__ __forceinline__ int grid_cur(const CaseView<T, R> &v, int64_t k) {
  const int launches = (v.n_sub + kSubstepBlock - 1) / kSubstepBlock;
  return ((launches + 1) & 1) ? (int)(k & 1) : 0;
}

// ---- K1: fused pull stream + BGK collide, Eq.(LBE) -------------------------
// A lane updates RPT rows of one lattice column: the pulls of all its rows
// are issued first, before the step's rectangle (a load that depends on the
// device step counter) is known; nodes inside the rectangle (unused and
// interpolation nodes) then carry their own values instead. Nodes a finer
// level covers, and the ring of a level fed by a coarser one, are skipped
// before any load.
template <class T, class R>
__device__ __forceinline__ bool static_skip(const CaseView<T, R> &v, int x, int y) {
  return (x > v.sx0 && x < v.sx1 && y > v.sy0 && y < v.sy1) ||
         (v.bc == 3 && (x == 0 || y == 0 || x == v.nx - 1 || y == v.ny - 1));
}

// a density that is not positive (or not a number) stops the case: bit 2 of
// its flag (bit 1: a non-finite force)
constexpr int kFlagForce = 1, kFlagDensity = 2, kFlagLocate = 4;  // bit 3: a lattice node off the grid
template <class R>
__device__ __forceinline__ void check_density(int *flag, R rho) {
  if (!(rho > R(0)) && flag) atomicOr(flag, kFlagDensity);
}

template <class T, class R, int RPT>
__device__ __forceinline__ void stream_collide_block(const CaseView<T, R> &v, const T *__restrict__ A,
                                                     T *__restrict__ B, const int64_t *k_at, int bx, int by) {
  const int x = v.wx0 + bx * blockDim.x + threadIdx.x;
  if (x >= v.wx0 + v.ww) return;
  const size_t plane = v.plane;
  const int y0 = v.wy0 + by * RPT, yend = v.wy0 + v.wh;
  R f[RPT][9];
#pragma unroll
  for (int r = 0; r < RPT; ++r)
    if (y0 + r < yend && !static_skip(v, x, y0 + r)) pull<T, R>(A, v.nx, v.ny, plane, v.bc, x, y0 + r, f[r]);
  int ix0 = 1, ix1 = 0, iy0 = 1, iy1 = 0;  // empty rectangle without a grid
  if (v.has_grid) {
    const StepParams &P = v.params[*k_at];
    ix0 = P.ix0, ix1 = P.ix1, iy0 = P.iy0, iy1 = P.iy1;
  }
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int y = y0 + r;
    if (y >= yend || static_skip(v, x, y)) continue;
    const size_t c = (size_t)y * v.nx + x;
    if (x >= ix0 && x <= ix1 && y >= iy0 && y <= iy1) {
#pragma unroll
      for (int q = 0; q < 9; ++q) B[q * plane + c] = A[q * plane + c];
      continue;
    }
    R e[9], rho, ux, uy;
    moments<R>(f[r], rho, ux, uy);
    check_density(v.flag, rho);
    equilibrium<R>(rho, ux, uy, e);
#pragma unroll
    for (int q = 0; q < 9; ++q) Stor<T>::st_stream(B, q * plane + c, q, fmad(-v.inv_tau, f[r][q] - e[q], f[r][q]));
  }
}

template <class T, class R>
__device__ __forceinline__ void interface_donors_block(const CaseView<T, R> &v, const T *__restrict__ A, int64_t k,
                                                       int bx);

// banded: workgroups are dealt to the eight XCDs in turn, so give each XCD
// a contiguous band of rows and the rows a pull shares with its neighbours
// stay in that XCD's L2 (less HBM traffic, though not less time here).
// ndon (a multiple of 8) leading workgroups compute the grid's interface
// donors from the same source lattice A instead (they read A only, which
// the stream-collide does not write), so the small donor pass hides in the
// HBM-bound one; the lattice workgroups keep their XCD assignment.
template <class T, class R, int RPT>
__global__ __launch_bounds__(256) void k_stream_collide(CaseView<T, R> v, int nbx, int nblocks, int banded,
                                                        int ndon) {
  const int b = (int)blockIdx.x - ndon;
  if (b < 0) {
    interface_donors_block<T, R>(v, v.A, *v.dk, blockIdx.x);
    return;
  }
  const int t = (banded && nblocks % 8 == 0) ? (b % 8) * (nblocks / 8) + (b / 8) : b;
  stream_collide_block<T, R, RPT>(v, v.A, v.B, v.dk, t % nbx, t / nbx);
}

// item = (case, column block, row group of RPT rows)
template <class T, class R, int RPT>
__global__ __launch_bounds__(256) void kb_stream_collide(const CaseView<T, R> *__restrict__ views,
                                                         const int4 *__restrict__ items) {
  const int4 it = items[blockIdx.x];
  const CaseView<T, R> &v = views[it.x];
  int64_t k;
  if (!batched_case(v, k)) return;
  stream_collide_block<T, R, RPT>(v, v.lat[k & 1], v.lat[(k + 1) & 1], v.dk, it.y, it.z);
}

// ---- K1 over two steps --------------------------------------------------------
// Nodes farther than the band from the fictitious rectangle never meet the
// grid coupling over two steps, so they advance t_k -> t_{k+2} in one
// launch: the first step (the same arithmetic as K1, rectangle nodes
// carrying their values) on the tile and a one-node ring around it, kept in
// LDS; the second step pulls from there, following the boundary rules of
// pull_source; it sees each first-step value as the stored lattice would
// hold it (rounded to the storage type). The band and one node around it
// also get t_{k+1} in B, from
// which the single-step kernel advances the band after the grid has written
// its interpolation nodes.
template <class T, class R>
//
// Tile order: with stagger >= 0 (and a tile count divisible by 8) the tiles
// are dealt to the eight XCDs (which take workgroups in turn) in contiguous
// runs of rows, so the rows a tile's ring shares with the tiles above and
// below are fetched into that XCD's L2 once; each XCD starts its run
// `stagger` tiles further along, so the eight XCDs do not stream from
// addresses a power of two apart (which share HBM channels). ndon leading
// workgroups compute the interface donors, as in k_stream_collide.
__global__ __launch_bounds__(512) void k_stream_collide2(CaseView<T, R> v, int tiles_x, int stagger, int ndon) {
  constexpr int TX = kTwoStepTX, TY = kTwoStepTY, NT = 512, LX = TX + 2, LY = TY + 2, LN = LX * LY;
  constexpr int P1 = (LN + NT - 1) / NT;
  static_assert(TX * TY == NT, "one output node per lane");
  __shared__ R s[9 * LN];
  const int nx = v.nx, ny = v.ny;
  const size_t plane = v.plane;
  int t = (int)blockIdx.x - ndon;
  if (t < 0) {
    interface_donors_block<T, R>(v, v.A, *v.dk, blockIdx.x);
    return;
  }
  const int ntiles = (int)gridDim.x - ndon;
  if (stagger >= 0 && ntiles % 8 == 0) {
    const int per = ntiles / 8, xcd = t % 8, i = t / 8;
    t = xcd * per + (i + xcd * stagger) % per;
  }
  const int tx0 = (t % tiles_x) * TX, ty0 = (t / tiles_x) * TY;
  R f[P1][9];
  int node[P1];
#pragma unroll
  for (int u = 0; u < P1; ++u) {
    const int i = threadIdx.x + u * NT;
    if (i < LN) {
      const int gx = ((tx0 - 1 + i % LX) % nx + nx) % nx, gy = ((ty0 - 1 + i / LX) % ny + ny) % ny;
      node[u] = gy * nx + gx;
      pull<T, R>(v.A, nx, ny, plane, v.bc, gx, gy, f[u]);
    }
  }
  int ix0 = 1, ix1 = 0, iy0 = 1, iy1 = 0;
  if (v.has_grid) {
    const StepParams &P = v.params[*v.dkl];
    ix0 = P.ix0, ix1 = P.ix1, iy0 = P.iy0, iy1 = P.iy1;
  }
#pragma unroll
  for (int u = 0; u < P1; ++u) {
    const int i = threadIdx.x + u * NT;
    if (i >= LN) continue;
    const int gx = node[u] % nx, gy = node[u] / nx;
    if (gx >= ix0 && gx <= ix1 && gy >= iy0 && gy <= iy1) {
#pragma unroll
      for (int q = 0; q < 9; ++q) f[u][q] = Stor<T>::ld(v.A, q * plane + node[u], q);
    } else {
      R e[9], rho, ux, uy;
      moments<R>(f[u], rho, ux, uy);
      equilibrium<R>(rho, ux, uy, e);
#pragma unroll
      for (int q = 0; q < 9; ++q) f[u][q] = fmad(-v.inv_tau, f[u][q] - e[q], f[u][q]);
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) s[q * LN + i] = f[u][q];
  }
  __syncthreads();
  const int ox = threadIdx.x % TX, oy = threadIdx.x / TX;
  const int x = tx0 + ox, y = ty0 + oy;
  if (x >= nx || y >= ny) return;
  const size_t c = (size_t)y * nx + x;
  const int l = (oy + 1) * LX + ox + 1;
  if (x >= v.bx0 - 1 && x <= v.bx1 + 1 && y >= v.by0 - 1 && y <= v.by1 + 1) {
    if (x >= ix0 && x <= ix1 && y >= iy0 && y <= iy1) {
#pragma unroll
      for (int q = 0; q < 9; ++q) v.B[q * plane + c] = v.A[q * plane + c];
    } else {
#pragma unroll
      for (int q = 0; q < 9; ++q) Stor<T>::st_stream(v.B, q * plane + c, q, s[q * LN + l]);
    }
    if (x >= v.bx0 && x <= v.bx1 && y >= v.by0 && y <= v.by1) return;
  }
  R g[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    int qs, xs, ys;
    pull_source(nx, ny, v.bc, x, y, q, qs, xs, ys);
    int lx = xs - (tx0 - 1), ly = ys - (ty0 - 1);  // tile coordinates, across a periodic seam too
    lx += lx < 0 ? nx : (lx >= LX ? -nx : 0);
    ly += ly < 0 ? ny : (ly >= LY ? -ny : 0);
    g[q] = Stor<T>::round_trip(s[qs * LN + ly * LX + lx], qs);  // as if stored at t_{k+1} and loaded
  }
  R e[9], rho, ux, uy;
  moments<R>(g, rho, ux, uy);
  check_density(v.flag, rho);
  equilibrium<R>(rho, ux, uy, e);
#pragma unroll
  for (int q = 0; q < 9; ++q) Stor<T>::st_stream(v.C, q * plane + c, q, fmad(-v.inv_tau, g[q] - e[q], g[q]));
}

// ---- K2: lattice interpolation nodes from the grid, Eq.(postcollision2_s) ----
// Targets: nodes inside the fictitious rectangle with a neighbour outside it
// (interpolation nodes), and nodes the moving rectangle uncovered since the
// previous step. Barycentric interpolation of rho, u and f^neq,u over the
// grid triangle at t_k; f^eq rebuilt from the interpolated moments.
template <class T, class R>
__device__ __forceinline__ void lattice_from_grid_block(const CaseView<T, R> &v, T *__restrict__ A,
                                                        const R *__restrict__ g, int64_t k, int bx, int by) {
  const StepParams &P = v.params[k];
  const int x = v.k2_x0 + bx * blockDim.x + threadIdx.x;
  const int y = min(P.iy0, P.piy0) + by;
  if (x >= v.k2_x0 + v.k2_w || y > max(P.iy1, P.piy1)) return;
  if (!from_grid_target(P, x, y)) return;
  int node[3];
  double lam[3];
  if (v.mesh) {
    if (mesh_locate(v.mg, (double)x - v.xc, (double)y - P.ybase, node, lam) < 0) {
      atomicOr(v.flag, kFlagLocate);  // the grid does not cover the node: the case stops
      return;
    }
  } else {
    const GridGeom gg{v.nux, v.nuy, v.h, v.xc, v.half_b, v.half_T, v.body, v.gx, v.gy};
    int ci, cj, tri;
    double a, b, dlam[3];
    lattice_node_cell(gg, P.ybase, x, y, ci, cj, a, b, tri);
    cell_triangle(ci, cj, v.nux, a, b, node, lam, dlam, tri);
  }
  R rho, ux, uy, fneq[9];
  grid_barycentric<R>(g, v.nnode, node, lam, rho, ux, uy, fneq);
  R e[9];
  equilibrium<R>(rho, ux, uy, e);
  const size_t plane = v.plane, c = (size_t)y * v.nx + x;
#pragma unroll
  for (int q = 0; q < 9; ++q) Stor<T>::st(A, q * plane + c, q, e[q] + v.g_post * fneq[q]);
}

template <class T, class R>
__global__ __launch_bounds__(256) void k_lattice_from_grid(CaseView<T, R> v, const R *__restrict__ g) {
  lattice_from_grid_block<T, R>(v, const_cast<T *>(v.A), g, *v.dk, blockIdx.x, blockIdx.y);
}

template <class T, class R>
__global__ __launch_bounds__(256) void kb_lattice_from_grid(const CaseView<T, R> *__restrict__ views,
                                                            const int4 *__restrict__ items) {
  const int4 it = items[blockIdx.x];
  const CaseView<T, R> &v = views[it.x];
  int64_t k;
  if (!batched_case(v, k)) return;
  lattice_from_grid_block<T, R>(v, v.lat[k & 1], v.grid[grid_cur(v, k)], k, it.y, it.z);
}

// ---- K4 prologue: structured-derived values at the grid's outer nodes ----------
// f* = f^eq,s + (1 - 1/(2 tau_s)) f^neq,s and f^neq* from the lattice at t_{k+1}
// (pre-collision), held over the n sub-steps (Eq.(postcollision2_u)). Four
// consecutive lanes take the four bilinear donors of one node and combine
// their weighted moments with two shuffles.
template <class T, class R>
__device__ __forceinline__ void interface_donors_block(const CaseView<T, R> &v, const T *__restrict__ A, int64_t k,
                                                       int bx) {
  const int gt = bx * blockDim.x + threadIdx.x;
  const int t = gt >> 2, d = gt & 3;
  const bool valid = t < v.n_iface;
  R acc[12];
#pragma unroll
  for (int r = 0; r < 12; ++r) acc[r] = R(0);
  int p = 0;
  if (valid) {
    const StepParams &P = v.params[k];
    p = v.iface[t];
    double X, Y;
    if (v.mesh) {
      X = v.xc + v.m_x[p];
      Y = P.ybase + v.m_y[p];
    } else {
      const int i = p % v.nux, j = p / v.nux;
      X = v.gx ? v.xc + v.gx[i] : v.xc + (double)(i - v.nux / 2) * v.h;
      Y = v.gy ? P.ybase + v.gy[j] : P.ybase + ((double)j - 0.5 * (double)(v.nuy - 1)) * v.h;
    }
    donor_corner<T, R>(A, v.nx, v.ny, v.plane, v.bc, X, Y, d, acc);
  }
#pragma unroll
  for (int r = 0; r < 12; ++r) {
    acc[r] += __shfl_xor(acc[r], 1, 64);
    acc[r] += __shfl_xor(acc[r], 2, 64);
  }
  if (!valid) return;
  R e[9];
  equilibrium<R>(acc[0], acc[1], acc[2], e);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    if ((q & 3) != d) continue;
    const R n = v.k_neq * acc[3 + q];
    v.star_n[(size_t)q * v.nnode + p] = n;
    v.star_f[(size_t)q * v.nnode + p] = e[q] + n;
  }
}

template <class T, class R>
__global__ __launch_bounds__(256) void k_interface_donors(CaseView<T, R> v) {
  interface_donors_block<T, R>(v, v.A, *v.dk, blockIdx.x);
}

template <class T, class R>
__global__ __launch_bounds__(256) void kb_interface_donors(const CaseView<T, R> *__restrict__ views,
                                                           const int4 *__restrict__ items) {
  const int4 it = items[blockIdx.x];
  const CaseView<T, R> &v = views[it.x];
  int64_t k;
  if (!batched_case(v, k)) return;
  interface_donors_block<T, R>(v, v.lat[k & 1], k, it.y);
}

// ---- K3/K4: sub-steps of the grid scheme ------------------------------------
// Eq.(ulbe) at discretization and wall nodes; Eq.(postcollision2_u) at the
// outer interpolation nodes, where the node itself and every interpolation
// neighbour contribute their structured-derived values. Wall nodes then take
// the lamina velocity while keeping density and non-equilibrium part.
//
// One launch advances `count` <= H sub-steps (temporal blocking). A
// workgroup owns a TX x TY tile and stages the tile plus an H-node halo in
// LDS, node-major: f and the three products rho u_a u_b of the node's
// moments (stride 13, odd, so wave64 reads of 64-bit values are free of bank
// conflicts). The collision sum needs f^neq = f - f^eq(rho, u) of every
// neighbour; since f^eq is linear in (rho, rho u, rho u u), the C-weighted
// sum of the neighbours' f^eq follows from the C-weighted sums of their f
// (which give sum C rho and sum C rho u) and of their rho u u, so a
// neighbour's f is read once for both the streaming and the collision sum
// and its f^neq is never stored. It also
// keeps the structured-derived values of nodes on the grid's outer ring and
// the stencil class and type of each node. Sub-step s updates the region
// grown by count-1-s around the tile, so after `count` sub-steps the tile is
// exact and only it is written back. In every sub-step the lanes are dealt
// afresh over that shrinking rectangle, so no wave works on nodes outside
// it; stencil coefficients are read from the class table (interior nodes
// share one class, so the reads are cache broadcasts). Tiles are dealt to
// the eight XCDs in contiguous bands.
constexpr int NS = 13;  // LDS doubles (or floats) per node: f[9], rho u_x u_x, rho u_x u_y, rho u_y u_y, pad

// the products rho u_x u_x, rho u_x u_y, rho u_y u_y of f's moments (the
// quadratic part of f^eq)
template <class R>
__device__ __forceinline__ void quad_moments(const R f[9], R P[3]) {
  R r, vx, vy;
  moments<R>(f, r, vx, vy);
  const R jx = r * vx, jy = r * vy;
  P[0] = jx * vx;
  P[1] = jx * vy;
  P[2] = jy * vy;
}

template <int TXv, int TYv, int H>
struct Region {
  static constexpr int TX = TXv, TY = TYv;
  static constexpr int RX = TX + 2 * H, RY = TY + 2 * H, RN = RX * RY;
  static constexpr int NRING = 2 * RX + 2 * RY;  // region nodes that can lie on the outer ring
  // nodes updated by the first sub-step of a full block
  static constexpr int MAXA = (TX + 2 * (H - 1)) * (TY + 2 * (H - 1));
};

// slot of region node (rx, ry) (global (gi, gj)) in the ring array, or -1
// when the node is not a grid node on the outer ring
template <class G>
__device__ __forceinline__ int ring_slot(int gi, int gj, int rx, int ry, int nux, int nuy) {
  if (gi < 0 || gj < 0 || gi >= nux || gj >= nuy) return -1;
  if (gj == 0) return rx;
  if (gj == nuy - 1) return G::RX + rx;
  if (gi == 0) return 2 * G::RX + ry;
  if (gi == nux - 1) return 2 * G::RX + G::RY + ry;
  return -1;
}

// DB: two copies of the region, so that a sub-step reads one and writes the
// other and a single barrier separates sub-steps
template <class R, class G, bool DB = false>
constexpr size_t substeps_lds_bytes() {
  return sizeof(R) * (size_t)(NS * G::RN * (DB ? 2 : 1) + NS * G::NRING) + sizeof(int) * (size_t)G::RN;
}
// the region is double-buffered when both copies fit a CU's LDS
template <class R, class G>
constexpr bool substeps_double_buffer() {
  return substeps_lds_bytes<R, G, true>() <= 160u * 1024u;
}

// Advances tile t of a grid by `count` sub-steps m0 .. m0+count-1 of step k.
template <class R, class G, int H, int NT, bool DB = false>
__device__ __forceinline__ void grid_substeps_block(
    const R *__restrict__ f, R *__restrict__ fout, const R *__restrict__ star_f, const R *__restrict__ star_n,
    const int *__restrict__ ncode, const GridClass<R> *__restrict__ tab, int nux, int nuy, int tiles_x, int t,
    R dt, R dt_tau, const R *__restrict__ uw, int64_t k, int n_sub, int m0, int count,
    R *__restrict__ tape, R *__restrict__ wtape, const int *__restrict__ widx, int nwall) {
  constexpr int TX = G::TX, TY = G::TY, RX = G::RX, RN = G::RN;
  constexpr int SPER = (RN + NT - 1) / NT;      // staging passes
  constexpr int PER = (G::MAXA + NT - 1) / NT;  // update passes
  extern __shared__ __align__(16) unsigned char lds_raw[];
  R *sl = reinterpret_cast<R *>(lds_raw);   // [RN][NS] grid f, rho u u (DB: two copies)
  constexpr int RING = NS * RN * (DB ? 2 : 1);  // offset of the ring values
  R *rl = sl + RING;                        // [NRING][NS] f*, rho* u* u* on the outer ring
  int *scode = reinterpret_cast<int *>(rl + NS * G::NRING);  // 4 * class + type, -1 outside the grid
  const int x0 = (t % tiles_x) * TX - H, y0 = (t / tiles_x) * TY - H;  // region origin
  const bool touches_ring = x0 <= 0 || y0 <= 0 || x0 + RX >= nux || y0 + G::RY >= nuy;
  const size_t N = (size_t)nux * nuy;
  // the lamina velocity of every sub-step of the launch, read up front: a
  // scalar load still in flight would hold up every later LDS wait
  R uwv[H];
#pragma unroll
  for (int sub = 0; sub < H; ++sub) uwv[sub] = sub < count ? uw[k * n_sub + m0 + sub] : R(0);

  // stage the region; a lane's loads are issued together
  {
    R v[SPER][9];
    bool inside[SPER];
#pragma unroll
    for (int u = 0; u < SPER; ++u) {
      const int idx = threadIdx.x + u * NT;
      const int gi = x0 + idx % RX, gj = y0 + idx / RX;
      const bool in = idx < RN && gi >= 0 && gi < nux && gj >= 0 && gj < nuy;
      inside[u] = in;
      const size_t p = in ? (size_t)gj * nux + gi : 0;
#pragma unroll
      for (int q = 0; q < 9; ++q) v[u][q] = in ? f[q * N + p] : R(0);
      if (idx < RN) scode[idx] = in ? ncode[p] : -1;
      if (touches_ring && in) {
        const int rs = ring_slot<G>(gi, gj, idx % RX, idx / RX, nux, nuy);
        if (rs >= 0) {
          R fs[9], P[3];
#pragma unroll
          for (int q = 0; q < 9; ++q) fs[q] = star_f[q * N + p];
          quad_moments<R>(fs, P);
#pragma unroll
          for (int q = 0; q < 9; ++q) rl[rs * NS + q] = fs[q];
#pragma unroll
          for (int a = 0; a < 3; ++a) rl[rs * NS + 9 + a] = P[a];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < SPER; ++u) {
      const int idx = threadIdx.x + u * NT;
      if (idx >= RN) continue;
      R P[3] = {R(0), R(0), R(0)};
      if (inside[u]) quad_moments<R>(v[u], P);
#pragma unroll
      for (int q = 0; q < 9; ++q) sl[idx * NS + q] = v[u][q];
#pragma unroll
      for (int a = 0; a < 3; ++a) sl[idx * NS + 9 + a] = P[a];
      if (DB && !inside[u])  // never written by a sub-step: zero in both copies
#pragma unroll
        for (int a = 0; a < NS; ++a) sl[NS * RN + idx * NS + a] = R(0);
    }
  }
  __syncthreads();

  // the node (region index) and code of pass u of a lane in sub-step sub
  auto lane_node = [&](int sub, int u, int &idx, int &code) {
    const int ex = max(count - 1 - sub, 0);  // region growth still exact after sub-step `sub`
    const int W = TX + 2 * ex, NA = sub < count ? W * (TY + 2 * ex) : 0, o = H - ex;
    const int j = threadIdx.x + u * NT;
    idx = j < NA ? (o + j / W) * RX + o + j % W : 0;
    code = j < NA ? scode[idx] : -1;
  };

  // Eq.(ulbe) at one node: streaming c_q . sum_s G_s f_q,s and collision
  // sum_s C_s f^neq_q,s = A_q - sum_s C_s f^eq_q(m_s), A_q = sum_s C_s f_q,s,
  // where sum_s C_s f^eq_q(m_s) = w_q (S_rho + 3 c_q.S_j + 4.5 c_q c_q : S_P
  // - 1.5 tr S_P) with S_rho = sum_q A_q, S_j = sum_q c_q A_q and S_P =
  // sum_s C_s (rho u u)_s. On the outer ring an interpolation node reads
  // structured-derived values instead (Eq.(postcollision2_u)). Absent
  // neighbours have zero weights.
  // Slots outside the mask M are known to carry zero weights and are skipped
  // (the same sums: a zero-weight term adds an exact zero).
  auto update_node = [&](auto mask, int idx, int code, const GridClass<R> &cl, int cur, R o9[9]) {
    constexpr int M = decltype(mask)::value;
    const int rx = idx % RX, ry = idx / RX;
    const int typ = code & 3;
    const int gi = x0 + rx, gj = y0 + ry;
    int row[NSLOT];
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
      if (!((M >> s) & 1)) continue;
      const int di = s % 3 - 1, dj = s / 3 - 1;
      row[s] = cur + (idx + dj * RX + di) * NS;
      if (typ == NODE_INTERFACE) {
        const int rs = ring_slot<G>(gi + di, gj + dj, rx + di, ry + dj, nux, nuy);
        if (rs >= 0) row[s] = RING + rs * NS;
      }
    }
    // out_q = f_q + dt c_q.(G f_q) - dt/tau (A_q - sum_s C_s f^eq_q(m_s)): the
    // part without the f^eq sum first, population by population, while the
    // sums S_rho and S_j accumulate; then the f^eq sum of every population
    R srho = R(0), sjx = R(0), sjy = R(0);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      R a = R(0), ax = R(0), ay = R(0);
#pragma unroll
      for (int s = 0; s < NSLOT; ++s) {
        if (!((M >> s) & 1)) continue;
        const R fq = sl[row[s] + q];
        a = fmad(cl.C[s], fq, a);
        if (CXd[q] != 0) ax = fmad(cl.Gx[s], fq, ax);
        if (CYd[q] != 0) ay = fmad(cl.Gy[s], fq, ay);
      }
      srho += a;
      if (CXd[q] != 0) sjx += R(CXd[q]) * a;
      if (CYd[q] != 0) sjy += R(CYd[q]) * a;
      o9[q] = fmad(-dt_tau, a, fmad(dt, R(CXd[q]) * ax + R(CYd[q]) * ay, sl[row[SELF_SLOT] + q]));
    }
    R pxx = R(0), pxy = R(0), pyy = R(0);
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
      if (!((M >> s) & 1)) continue;
      const R c = cl.C[s];
      pxx = fmad(c, sl[row[s] + 9], pxx);
      pxy = fmad(c, sl[row[s] + 10], pxy);
      pyy = fmad(c, sl[row[s] + 11], pyy);
    }
    const R base = fmad(R(-1.5), pxx + pyy, srho);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const R cx = R(CXd[q]), cy = R(CYd[q]);
      const R cu = cx * sjx + cy * sjy;
      const R cc = (cx * cx) * pxx + (R(2) * cx * cy) * pxy + (cy * cy) * pyy;
      o9[q] = fmad(dt_tau * wgt<R>(q), fmad(R(4.5), cc, fmad(R(3), cu, base)), o9[q]);
    }
  };
  // copy a sub-step reads (offset into the LDS values); DB: the other copy
  // receives its results
  auto copy_of = [&](int sub) { return DB ? (sub & 1) * NS * RN : 0; };
  // the node codes never change within a launch: each sub-step's are read
  // before the barrier that ends the previous one
  int nidx[PER], ncd[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) lane_node(0, u, nidx[u], ncd[u]);
#pragma unroll
  for (int sub = 0; sub < H; ++sub) {
    if (sub >= count) break;
    const R uw_now = uwv[sub];
    const int cur = copy_of(sub), nxt = copy_of(sub + 1);
    R out[PER][9];
    int sidx[PER], scd[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      sidx[u] = nidx[u];
      scd[u] = ncd[u];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = sidx[u], code = scd[u];
#pragma unroll
      for (int q = 0; q < 9; ++q) out[u][q] = R(0);
      if (__ballot(code >= 0) == 0) continue;  // nothing to update in this wave
      // a wave whose nodes all lack the same two diagonal neighbours (the
      // interior of either half of a split-quad grid) skips those slots;
      // with one node per lane only, to bound the code size
      int zd = 0;
      if constexpr (PER == 1) {
        const int z = code >= 0 ? (code >> 2) & 3 : kZeroDiag26 | kZeroDiag08;
        zd = __ballot(!(z & kZeroDiag26)) == 0 ? kZeroDiag26 : __ballot(!(z & kZeroDiag08)) == 0 ? kZeroDiag08 : 0;
      }
      if (code < 0) continue;
      const GridClass<R> &cl = tab[code >> 4];
      if (zd == kZeroDiag26)
        update_node(std::integral_constant<int, 0x1FF & ~(1 << 2 | 1 << 6)>{}, idx, code, cl, cur, out[u]);
      else if (zd == kZeroDiag08)
        update_node(std::integral_constant<int, 0x1FF & ~(1 << 0 | 1 << 8)>{}, idx, code, cl, cur, out[u]);
      else
        update_node(std::integral_constant<int, 0x1FF>{}, idx, code, cl, cur, out[u]);
      if ((code & 3) == NODE_WALL) {
        // wall nodes: impose the lamina velocity, keep rho and f^neq
        const int rx = idx % RX, ry = idx / RX;
        R e[9], ew[9], r, vx, vy;
        moments<R>(out[u], r, vx, vy);
        if (wtape && rx >= H && rx < H + TX && ry >= H && ry < H + TY) {
          // taped for the adjoint: the moments before the velocity is imposed
          R *wt = wtape + (size_t)(m0 + sub) * 3 * nwall;
          const int w = widx[(size_t)(y0 + ry) * nux + (x0 + rx)];
          wt[w] = r;
          wt[nwall + w] = vx;
          wt[2 * nwall + w] = vy;
        }
        equilibrium<R>(r, vx, vy, e);
        equilibrium<R>(r, R(0), uw_now, ew);
#pragma unroll
        for (int q = 0; q < 9; ++q) out[u][q] = ew[q] + (out[u][q] - e[q]);
      }
      if (DB) {  // the other copy: written at once, read after the barrier
        R P[3];
        quad_moments<R>(out[u], P);
#pragma unroll
        for (int q = 0; q < 9; ++q) sl[nxt + idx * NS + q] = out[u][q];
#pragma unroll
        for (int a = 0; a < 3; ++a) sl[nxt + idx * NS + 9 + a] = P[a];
      }
    }
    if (!DB) {  // one copy: every read of the sub-step ends before the writes
      __syncthreads();
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = sidx[u], code = scd[u];
        if (code < 0) continue;
        R P[3];
        quad_moments<R>(out[u], P);
#pragma unroll
        for (int q = 0; q < 9; ++q) sl[idx * NS + q] = out[u][q];
#pragma unroll
        for (int a = 0; a < 3; ++a) sl[idx * NS + 9 + a] = P[a];
      }
    }
    if (sub + 1 < count)
#pragma unroll
      for (int u = 0; u < PER; ++u) lane_node(sub + 1, u, nidx[u], ncd[u]);
    __syncthreads();
    // the tile is exact after every sub-step: a tape keeps the intermediate ones
    if (tape && sub + 1 < count) {
      R *dst = tape + (size_t)(m0 + sub + 1) * 9 * N;
      for (int jn = threadIdx.x; jn < TX * TY; jn += NT) {
        const int rx = H + jn % TX, ry = H + jn / TX;
        const int gi = x0 + rx, gj = y0 + ry;
        if (gi >= nux || gj >= nuy) continue;
        const int ci = ry * RX + rx;
        const size_t p = (size_t)gj * nux + gi;
#pragma unroll
        for (int q = 0; q < 9; ++q) dst[q * N + p] = sl[nxt + ci * NS + q];
      }
    }
  }

  // the tile is exact: write it back
  const int last = copy_of(count);
  for (int j = threadIdx.x; j < TX * TY; j += NT) {
    const int rx = H + j % TX, ry = H + j / TX;
    const int gi = x0 + rx, gj = y0 + ry;
    if (gi >= nux || gj >= nuy) continue;
    const int ci = ry * RX + rx;
    const size_t p = (size_t)gj * nux + gi;
#pragma unroll
    for (int q = 0; q < 9; ++q) fout[q * N + p] = sl[last + ci * NS + q];
  }
}

// Variants of the sub-step kernel: tile shape and workgroup size (one lane
// per region node while staging). Variant 3's LDS fits two workgroups on a
// CU in FP64 and more in FP32 (many small grids).
template <int TXv, int TYv, int NTv, int Hv = kSubstepBlock>
struct SubstepShape {
  using G = Region<TXv, TYv, Hv>;
  static constexpr int NT = NTv;
  static constexpr int H = Hv;  // sub-steps per launch, and the halo width
};
template <int V>
struct SubstepVariant;
template <> struct SubstepVariant<0> : SubstepShape<16, 16, 576> {};
template <> struct SubstepVariant<1> : SubstepShape<32, 8, 640> {};
template <> struct SubstepVariant<2> : SubstepShape<64, 4, 896> {};
template <> struct SubstepVariant<3> : SubstepShape<16, 8, 384> {};
template <> struct SubstepVariant<4> : SubstepShape<8, 8, 64> {};
template <> struct SubstepVariant<5> : SubstepShape<16, 8, 128> {};
template <> struct SubstepVariant<6> : SubstepShape<16, 16, 256> {};
template <> struct SubstepVariant<7> : SubstepShape<8, 4, 64> {};
template <> struct SubstepVariant<8> : SubstepShape<32, 8, 256, 1> {};
template <> struct SubstepVariant<9> : SubstepShape<16, 16, 256, 1> {};
template <> struct SubstepVariant<10> : SubstepShape<32, 8, 384, 2> {};

template <class R, int V>
__global__ __launch_bounds__(SubstepVariant<V>::NT) void k_grid_substeps(
    const R *__restrict__ f, R *__restrict__ fout, const R *__restrict__ star_f, const R *__restrict__ star_n,
    const int *__restrict__ ncode, const GridClass<R> *__restrict__ tab, int nux, int nuy, int tiles_x, int ntiles,
    R dt, R dt_tau, const R *__restrict__ uw, const int64_t *__restrict__ dk, int n_sub, int m0, int count,
    R *__restrict__ tape, R *__restrict__ wtape, const int *__restrict__ widx, int nwall) {
  using SV = SubstepVariant<V>;
  const int b = blockIdx.x;  // tiles are dealt to the eight XCDs in contiguous bands
  const int t = (ntiles % 8 == 0) ? (b % 8) * (ntiles / 8) + (b / 8) : b;
  grid_substeps_block<R, typename SV::G, SV::H, SV::NT, substeps_double_buffer<R, typename SV::G>()>(
      f, fout, star_f, star_n, ncode, tab, nux, nuy, tiles_x, t, dt, dt_tau, uw, *dk, n_sub, m0, count, tape, wtape,
      widx, nwall);
}

// launch m0 / kSubstepBlock of a batched step: item = (case, tile)
template <class T, class R, int V>
__global__ __launch_bounds__(SubstepVariant<V>::NT) void kb_grid_substeps(const CaseView<T, R> *__restrict__ views,
                                                                          const int4 *__restrict__ items, int m0) {
  using SV = SubstepVariant<V>;
  const int4 it = items[blockIdx.x];
  const CaseView<T, R> &v = views[it.x];
  int64_t k;
  if (!batched_case(v, k)) return;
  const int cur = grid_cur(v, k), i = m0 / kSubstepBlock;
  const int tiles_x = (v.nux + SV::G::TX - 1) / SV::G::TX;
  grid_substeps_block<R, typename SV::G, kSubstepBlock, SV::NT>(
      v.grid[cur ^ (i & 1)], v.grid[cur ^ ((i + 1) & 1)], v.star_f, v.star_n, v.ncode, v.tab, v.nux, v.nuy, tiles_x,
      it.y, v.dt_u, v.dt_over_tau_u, v.uw, k, v.n_sub, m0, min(kSubstepBlock, v.n_sub - m0), nullptr, nullptr,
      nullptr, 0);
}


// ---- K3/K4 on an unstructured grid -------------------------------------------
// One sub-step per launch, one node per lane. The node's stencil entries are
// read from the grid buffer (an interface node reads the structured-derived
// values for itself and its interface neighbours, Eq.(postcollision2_u)),
// and the update is that of the split-quad kernel: streaming c_q.(G f_q),
// and the collision sum of f^neq from the C-weighted sums of f and of
// rho u u (f^eq being linear in rho, rho u and rho u u), then the lamina
// velocity at wall nodes.
// small workgroups: a grid of some ten thousand nodes still spreads over
// every CU
constexpr int kMeshThreads = 64;
template <class T, class R>
__global__ __launch_bounds__(kMeshThreads) void k_mesh_substep(CaseView<T, R> v, const R *__restrict__ f,
                                                               R *__restrict__ fout, int m) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= v.nnode) return;
  const int64_t k = *v.dk;
  const size_t N = (size_t)v.nnode;
  const int typ = v.m_type[p];
  const bool iface = typ == NODE_INTERFACE;
  R a[9], ax[9], ay[9], self[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) a[q] = ax[q] = ay[q] = self[q] = R(0);
  R pxx = R(0), pxy = R(0), pyy = R(0);
  const int e0 = v.m_row[p], e1 = v.m_row[p + 1];
  for (int e = e0; e < e1; ++e) {
    const int nb = v.m_col[e];
    const R *src = (iface && v.m_type[nb] == NODE_INTERFACE) ? v.star_f : f;
    R fq[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) fq[q] = src[q * N + nb];
    if (e == e0)  // the node itself comes first
#pragma unroll
      for (int q = 0; q < 9; ++q) self[q] = fq[q];
    const R c = v.m_C[e], gx = v.m_Gx[e], gy = v.m_Gy[e];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      a[q] = fmad(c, fq[q], a[q]);
      if (CXd[q] != 0) ax[q] = fmad(gx, fq[q], ax[q]);
      if (CYd[q] != 0) ay[q] = fmad(gy, fq[q], ay[q]);
    }
    R P[3];
    quad_moments<R>(fq, P);
    pxx = fmad(c, P[0], pxx);
    pxy = fmad(c, P[1], pxy);
    pyy = fmad(c, P[2], pyy);
  }
  const R dt = v.dt_u, dt_tau = v.dt_over_tau_u;
  R srho = R(0), sjx = R(0), sjy = R(0), out[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    srho += a[q];
    if (CXd[q] != 0) sjx += R(CXd[q]) * a[q];
    if (CYd[q] != 0) sjy += R(CYd[q]) * a[q];
    out[q] = fmad(-dt_tau, a[q], fmad(dt, R(CXd[q]) * ax[q] + R(CYd[q]) * ay[q], self[q]));
  }
  const R base = fmad(R(-1.5), pxx + pyy, srho);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const R cx = R(CXd[q]), cy = R(CYd[q]);
    const R cu = cx * sjx + cy * sjy;
    const R cc = (cx * cx) * pxx + (R(2) * cx * cy) * pxy + (cy * cy) * pyy;
    out[q] = fmad(dt_tau * wgt<R>(q), fmad(R(4.5), cc, fmad(R(3), cu, base)), out[q]);
  }
  if (typ == NODE_WALL) {  // impose the lamina velocity, keep rho and f^neq
    R e[9], ew[9], r, vx, vy;
    moments<R>(out, r, vx, vy);
    equilibrium<R>(r, vx, vy, e);
    R uy = v.uw[k * v.n_sub + m];
    if (v.deform) uy = uy + v.uwb[k * v.n_sub + m] * v.m_sx[p];  // the wall's own bending velocity
    equilibrium<R>(r, R(0), uy, ew);
#pragma unroll
    for (int q = 0; q < 9; ++q) out[q] = ew[q] + (out[q] - e[q]);
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) fout[q * N + p] = out[q];
}

// ---- geometry of a bending unstructured grid ---------------------------------
// The extension to deformable bodies (Sec. Conclusions): node p of the
// reference triangulation sits at local y = yref_p + prof_p beta_k during
// step k. One launch at the start of the step rebuilds what depends on the
// configuration: lanes [0, nnode) the stencil weights of one node each,
// lanes [nnode, nnode + ntri) the vertex y of one triangle each (point
// location), the remaining lanes one wall edge each (length and unit normal
// toward the triangle's third vertex, out of the body). Node positions are
// rounded as a separate product and sum.
//
// A node's weights are the median-dual ones of the host assembly: over the
// triangles around it, V = sum |T|/3, C gains |T| 11/54 for the node itself
// and |T| 7/108 for each other vertex, and the gradient weight of vertex a,
// -(|T|/3) grad(phi_a), is the edge opposite a turned by 90 degrees over 6
// (no division). Each lane sums into its own column of LDS, one slot per
// stencil entry; a node with more than kDeformSlots entries takes the
// per-entry loop instead.
constexpr int kDeformThreads = 64, kDeformSlots = 16;
template <class R>
__global__ __launch_bounds__(kDeformThreads) void k_mesh_deform(MeshDeformView<R> g) {
  __shared__ double acc[kDeformSlots * 3][kDeformThreads];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x;
  const double beta = g.params[*g.dk].beta;
  auto ynode = [&](int n) { return __dadd_rn(g.yref[n], __dmul_rn(g.prof[n], beta)); };
  if (i < g.nnode) {
    const int p = i, t0 = g.trow[p], t1 = g.trow[p + 1], e0 = g.row[p], ne = g.row[p + 1] - e0;
    if (ne <= kDeformSlots) {
      for (int u = 0; u < ne; ++u) acc[3 * u][lane] = acc[3 * u + 1][lane] = acc[3 * u + 2][lane] = 0.0;
      double V = 0.0;
      for (int j = t0; j < t1; ++j) {
        const int packed = g.tslot[j];
        const int *v = g.tri + 3 * (size_t)g.tlist[j];
        double qx[3], qy[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
          qx[u] = g.x[v[u]];
          qy[u] = ynode(v[u]);
        }
        const double area = 0.5 * ((qx[1] - qx[0]) * (qy[2] - qy[0]) - (qx[2] - qx[0]) * (qy[1] - qy[0]));
        V += area / 3.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int ab = a == 2 ? 0 : a + 1, ac = a == 0 ? 2 : a - 1;
          const int slot = (packed >> (10 * a)) & 1023;
          acc[3 * slot][lane] += area * (slot == 0 ? 11.0 / 54.0 : 7.0 / 108.0);
          acc[3 * slot + 1][lane] += (qy[ac] - qy[ab]) / 6.0;
          acc[3 * slot + 2][lane] += (qx[ab] - qx[ac]) / 6.0;
        }
      }
      for (int u = 0; u < ne; ++u) {
        g.C[e0 + u] = (R)(acc[3 * u][lane] / V);
        g.Gx[e0 + u] = (R)(acc[3 * u + 1][lane] / V);
        g.Gy[e0 + u] = (R)(acc[3 * u + 2][lane] / V);
      }
      return;
    }
    double V = 0.0;
    for (int j = t0; j < t1; ++j) {
      const int *v = g.tri + 3 * (size_t)g.tlist[j];
      const double x0 = g.x[v[0]], x1 = g.x[v[1]], x2 = g.x[v[2]];
      const double y0 = ynode(v[0]), y1 = ynode(v[1]), y2 = ynode(v[2]);
      V += 0.5 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0)) / 3.0;
    }
    for (int slot = 0; slot < ne; ++slot) {
      double C = 0.0, Gx = 0.0, Gy = 0.0;
      for (int j = t0; j < t1; ++j) {
        const int packed = g.tslot[j];
        int a = -1;
#pragma unroll
        for (int u = 0; u < 3; ++u)
          if (((packed >> (10 * u)) & 1023) == slot) a = u;
        if (a < 0) continue;
        const int *v = g.tri + 3 * (size_t)g.tlist[j];
        double qx[3], qy[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
          qx[u] = g.x[v[u]];
          qy[u] = ynode(v[u]);
        }
        const double area = 0.5 * ((qx[1] - qx[0]) * (qy[2] - qy[0]) - (qx[2] - qx[0]) * (qy[1] - qy[0]));
        const int ab = a == 2 ? 0 : a + 1, ac = a == 0 ? 2 : a - 1;
        C += area * (slot == 0 ? 11.0 / 54.0 : 7.0 / 108.0);
        Gx += (qy[ac] - qy[ab]) / 6.0;
        Gy += (qx[ab] - qx[ac]) / 6.0;
      }
      g.C[e0 + slot] = (R)(C / V);
      g.Gx[e0 + slot] = (R)(Gx / V);
      g.Gy[e0 + slot] = (R)(Gy / V);
    }
    return;
  }
  const int t = i - g.nnode;
  if (t < g.ntri) {
#pragma unroll
    for (int a = 0; a < 3; ++a) g.txy[6 * (size_t)t + 2 * a + 1] = ynode(g.tri[3 * (size_t)t + a]);
    return;
  }
  const int w = t - g.ntri;
  if (w >= g.nwall) return;
  WallEdge &we = g.wall[w];
  const int o = g.wall_o[w];
  const double ya = ynode(we.a);
  const double ex = g.x[we.b] - g.x[we.a], ey = ynode(we.b) - ya;
  const double len = sqrt(ex * ex + ey * ey);
  double nx = -ey / len, ny = ex / len;
  if (nx * (g.x[o] - g.x[we.a]) + ny * (ynode(o) - ya) < 0.0) {
    nx = -nx;
    ny = -ny;
  }
  we.nx = nx;
  we.ny = ny;
  we.len = len;
}

// ---- K5: move the grid from y_k to y_{k+1} and refill it ---------------------
// Each non-wall node is located, at its new position, in the grid of t_k:
// inside a triangle -> type 3 (barycentric interpolation of f); inside the
// old lamina -> type 2 (keep f); otherwise -> type 1 (bilinear lattice
// donors, f^neq,u = (1 - 1/(2 tau_s)) f^neq,s, Eq.(continuity_stresses)).
// Wall nodes keep f (their velocity is imposed during the sub-steps).
template <class T, class R>
__device__ __forceinline__ void refill_block(const CaseView<T, R> &v, const T *__restrict__ A,
                                             const R *__restrict__ fo, R *__restrict__ fn, int64_t k, int bx) {
  const int p = bx * blockDim.x + threadIdx.x;
  if (p >= v.nnode) return;
  const size_t N = (size_t)v.nnode;
  R out[9];
  if ((v.mesh ? v.m_type[p] : (v.ncode[p] & 3)) == NODE_WALL) {
#pragma unroll
    for (int q = 0; q < 9; ++q) fn[q * N + p] = fo[q * N + p];
    return;
  }
  const StepParams &P = v.params[k];
  int node[3];
  double lam[3];
  RefillCell rc;
  double X, Ynew;
  if (v.mesh) {
    // the node's new position in the grid of t_k; not in any triangle:
    // inside the old lamina (type 2) or outside the old grid (type 1)
    // (a bending grid: the node's own new position, and the old lamina's
    // centreline beta_k (2x/b)^2 under it)
    X = v.xc + v.m_x[p];
    Ynew = P.ybase1 + (v.deform ? __dadd_rn(v.m_yref[p], __dmul_rn(v.m_prof[p], P.beta1)) : v.m_y[p]);
    const double xl = X - v.xc, yl = Ynew - P.ybase;
    double yb = 0.0;
    if (v.deform) {
      const double r = xl / v.half_b;
      yb = __dmul_rn(P.beta, __dmul_rn(r, r));
    }
    rc.kind = mesh_locate(v.mg, xl, yl, node, lam) >= 0 ? 3
              : (v.body && fabs(xl) < v.half_b && fabs(yl - yb) < v.half_T) ? 2 : 1;
  } else {
    const int i = p % v.nux, j = p / v.nux;
    const GridGeom gg{v.nux, v.nuy, v.h, v.xc, v.half_b, v.half_T, v.body, v.gx, v.gy};
    rc = refill_cell(gg, P.ybase, P.ybase1, i, j);
    X = v.gx ? v.xc + v.gx[i] : v.xc + (double)(i - v.nux / 2) * v.h;
    Ynew = v.gy ? P.ybase1 + v.gy[j] : P.ybase1 + ((double)j - 0.5 * (double)(v.nuy - 1)) * v.h;
    if (rc.kind == 3) {
      double dlam[3];
      cell_triangle(rc.ci, rc.cj, v.nux, rc.a, rc.b, node, lam, dlam, rc.tri);
    }
  }
  if (rc.kind == 3) {
#pragma unroll
    for (int q = 0; q < 9; ++q)
      out[q] = R(lam[0]) * fo[q * N + node[0]] + R(lam[1]) * fo[q * N + node[1]] + R(lam[2]) * fo[q * N + node[2]];
  } else if (rc.kind == 2) {
#pragma unroll
    for (int q = 0; q < 9; ++q) out[q] = fo[q * N + p];
    atomicAdd(&v.counts[1], 1ull);
  } else {
    R rho, ux, uy, fneq[9], e[9];
    lattice_bilinear<T, R>(A, v.nx, v.ny, v.plane, v.bc, X, Ynew, rho, ux, uy, fneq);
    equilibrium<R>(rho, ux, uy, e);
#pragma unroll
    for (int q = 0; q < 9; ++q) out[q] = e[q] + v.k_neq * fneq[q];
    atomicAdd(&v.counts[0], 1ull);
  }
  R rho = R(0);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    fn[q * N + p] = out[q];
    rho += out[q];
  }
  check_density(v.flag, rho);
}

template <class T, class R>
__global__ __launch_bounds__(256) void k_refill(CaseView<T, R> v, const R *__restrict__ fo, R *__restrict__ fn) {
  refill_block<T, R>(v, v.A, fo, fn, *v.dk, blockIdx.x);
}

template <class T, class R>
__global__ __launch_bounds__(256) void kb_refill(const CaseView<T, R> *__restrict__ views,
                                                 const int4 *__restrict__ items) {
  const int4 it = items[blockIdx.x];
  const CaseView<T, R> &v = views[it.x];
  int64_t k;
  if (!batched_case(v, k)) return;
  const int cur = grid_cur(v, k), L = (v.n_sub + kSubstepBlock - 1) / kSubstepBlock;
  refill_block<T, R>(v, v.lat[k & 1], v.grid[cur ^ (L & 1)], v.grid[cur ^ ((L + 1) & 1)], k, it.y);
}

// ---- K6: force on the lamina, then advance the step counter ------------------
// Traction -p' n + sigma' n on each wall edge (trapezoid rule), p' = c_s^2
// (rho - 1), sigma'_ab = -sum_i c_ia c_ib f_i^neq; FP64 accumulation over 256
// virtual lanes (lane l takes edges l, l + 256, ...), a wave64 shuffle
// reduction per group of 64 and one LDS pass across the four groups, so the
// sum is rounded the same way whatever the workgroup width (a multiple of
// 64, at most 256).
constexpr int kForceLanes = 256;
template <class R>
__device__ __forceinline__ void force_block(const R *__restrict__ f, const WallEdge *__restrict__ wall,
                                            int n_wall_edges, int nnode, int64_t *dk, double *hist, int *flag,
                                            const MotionCtx &mot = MotionCtx{}, StepParams *P = nullptr,
                                            R *uw = nullptr, int n_sub = 0, int advance = 1) {
  __shared__ double red[2][kForceLanes / 64];
  const int lane = threadIdx.x & 63;
  for (int vw = threadIdx.x >> 6; vw < kForceLanes / 64; vw += blockDim.x >> 6) {
    double Fx = 0.0, Fy = 0.0;
    for (int e = vw * 64 + lane; e < n_wall_edges; e += kForceLanes) {
      const WallEdge w = wall[e];
      double tx = 0.0, ty = 0.0;
      for (int s = 0; s < 2; ++s) {
        const int p = s ? w.b : w.a;
        R fp[9], eq[9], r, vx, vy;
#pragma unroll
        for (int q = 0; q < 9; ++q) fp[q] = f[(size_t)q * nnode + p];
        moments<R>(fp, r, vx, vy);
        equilibrium<R>(r, vx, vy, eq);
        double sxx = 0.0, sxy = 0.0, syy = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          const double fn = (double)fp[q] - (double)eq[q];
          sxx -= double(CXd[q] * CXd[q]) * fn;
          sxy -= double(CXd[q] * CYd[q]) * fn;
          syy -= double(CYd[q] * CYd[q]) * fn;
        }
        const double pp = ((double)r - 1.0) / 3.0;
        tx += -pp * w.nx + sxx * w.nx + sxy * w.ny;
        ty += -pp * w.ny + sxy * w.nx + syy * w.ny;
      }
      Fx += 0.5 * w.len * tx;
      Fy += 0.5 * w.len * ty;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      Fx += __shfl_xor(Fx, o, 64);
      Fy += __shfl_xor(Fy, o, 64);
    }
    if (lane == 0) {
      red[0][vw] = Fx;
      red[1][vw] = Fy;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i < kForceLanes / 64; ++i) {
      sx += red[0][i];
      sy += red[1][i];
    }
    const int64_t k = *dk;
    hist[2 * k] = sx;
    hist[2 * k + 1] = sy;
    if (!isfinite(sx) || !isfinite(sy)) atomicOr(flag, kFlagForce);
    if (mot.on) {
      // semi-implicit Euler, Delta t = 1: v_{k+1} from the force at t_{k+1},
      // then y_{k+1} = y_k + v_{k+1}; a state leaving |y| <= y_max or
      // |v| < 1 stops the case (flag) and the motion is frozen, so every
      // table stays inside the bounds the lattice was checked for
      const double y = mot.state[2 * k], vel = mot.state[2 * k + 1];
      const double acc = (sy - mot.K * y - mot.C * vel) / mot.M;
      double v1 = vel + acc, y1 = y + v1;
      if (!(fabs(y1) <= mot.y_max) || !(fabs(v1) < 1.0)) {
        atomicOr(flag, kFlagForce);
        y1 = y;
        v1 = 0.0;
      }
      mot.state[2 * (k + 1)] = y1;
      mot.state[2 * (k + 1) + 1] = v1;
      StepParams &Pk = P[k];
      Pk.y1 = y1;
      Pk.ybase1 = mot.yc + y1;
      if (k + 1 <= mot.cap) {
        StepParams &Pn = P[k + 1];
        Pn.y = y1;
        Pn.ybase = mot.yc + y1;
        Pn.ix0 = Pk.ix0;
        Pn.ix1 = Pk.ix1;
        Pn.iy0 = (int)ceil(((mot.yc + y1) + mot.c0) + mot.margin);
        Pn.iy1 = (int)floor(((mot.yc + y1) + mot.c1) - mot.margin);
        Pn.pix0 = Pk.ix0;
        Pn.pix1 = Pk.ix1;
        Pn.piy0 = Pk.iy0;
        Pn.piy1 = Pk.iy1;
      }
      if (k + 1 < mot.cap)
        for (int m = 0; m < n_sub; ++m) uw[(k + 1) * n_sub + m] = (R)v1;
    }
    if (advance) *dk = k + 1;
  }
}

__global__ void k_copy_step(const int64_t *from, int64_t *to) {
  if (threadIdx.x == 0) *to = *from;
}

__global__ void k_advance_step(int64_t *dk) {
  if (threadIdx.x == 0) *dk = *dk + 1;
}

template <class R>
__global__ __launch_bounds__(256) void k_force(const R *__restrict__ f, const WallEdge *__restrict__ wall,
                                               int n_wall_edges, int nnode, int64_t *dk, double *hist, int *flag,
                                               MotionCtx mot, StepParams *P, R *uw, int n_sub, int advance) {
  force_block<R>(f, wall, n_wall_edges, nnode, dk, hist, flag, mot, P, uw, n_sub, advance);
}

// Refill and force of one case in one launch: workgroup 0 computes the
// force of t_{k+1} on the grid before the refill, the others refill it.
// Every workgroup reads the step counter first and counts itself done at
// its end; the last one advances the counter (and clears the count for the
// next launch), so no workgroup can read the advanced step.
template <class T, class R>
__global__ __launch_bounds__(256) void k_refill_force(CaseView<T, R> v, const R *__restrict__ fo,
                                                      R *__restrict__ fn, unsigned *done) {
  __shared__ int64_t k_s;
  if (threadIdx.x == 0) k_s = *v.dk;
  __syncthreads();
  const int64_t k = k_s;
  if (blockIdx.x == 0)
    force_block<R>(fo, v.wall, v.n_wall_edges, v.nnode, v.dk, v.hist, v.flag, MotionCtx{}, nullptr, nullptr, 0,
                   0);
  else
    refill_block<T, R>(v, v.A, fo, fn, k, blockIdx.x - 1);
  __syncthreads();
  // the counter was read (into k) before this point; the next launch sees
  // the advanced counter and the cleared count at the kernel boundary
  if (threadIdx.x == 0) {
    if (atomicAdd(done, 1u) == gridDim.x - 1) {
      *done = 0u;
      *v.dk = k + 1;
    }
  }
}

// one workgroup per case: item = (case)
template <class T, class R>
__global__ __launch_bounds__(256) void kb_force(const CaseView<T, R> *__restrict__ views,
                                                const int4 *__restrict__ items) {
  const int4 it = items[blockIdx.x];
  const CaseView<T, R> &v = views[it.x];
  int64_t k;
  if (!batched_case(v, k)) return;
  const int cur = grid_cur(v, k), L = (v.n_sub + kSubstepBlock - 1) / kSubstepBlock;
  force_block<R>(v.grid[cur ^ (L & 1)], v.wall, v.n_wall_edges, v.nnode, v.dk, v.hist, v.flag);
}

// ---- persistent case-batched steps -------------------------------------------
// One cooperative launch advances the running cases of a batch by `steps`
// steps: every workgroup walks the phases of a step in their order (lattice
// interpolation nodes, stream-collide, donors, the sub-step blocks, refill,
// force), taking every gridDim-th work item of a phase, and the whole grid
// meets at a barrier after each phase, where the other path ends a launch.
// The work items and their block functions are those of the kb_* kernels,
// built for workgroups of the sub-step variant's width.
template <class T, class R, int V>
__device__ __forceinline__ void batch_item(const CaseView<T, R> *__restrict__ views, int4 it, int which, int m0) {
  using SV = SubstepVariant<V>;
  const CaseView<T, R> &v = views[it.x];
  int64_t k;
  if (!batched_case(v, k)) return;
  const int cur = grid_cur(v, k), L = (v.n_sub + kSubstepBlock - 1) / kSubstepBlock;
  switch (which) {
    case (int)BatchKernel::LatticeFromGrid:
      lattice_from_grid_block<T, R>(v, v.lat[k & 1], v.grid[cur], k, it.y, it.z);
      break;
    case (int)BatchKernel::StreamCollide:
      stream_collide_block<T, R, 1>(v, v.lat[k & 1], v.lat[(k + 1) & 1], v.dk, it.y, it.z);
      break;
    case (int)BatchKernel::InterfaceDonors:
      interface_donors_block<T, R>(v, v.lat[k & 1], k, it.y);
      break;
    case (int)BatchKernel::GridSubsteps: {
      const int i = m0 / kSubstepBlock;
      const int tiles_x = (v.nux + SV::G::TX - 1) / SV::G::TX;
      grid_substeps_block<R, typename SV::G, kSubstepBlock, SV::NT>(
          v.grid[cur ^ (i & 1)], v.grid[cur ^ ((i + 1) & 1)], v.star_f, v.star_n, v.ncode, v.tab, v.nux, v.nuy,
          tiles_x, it.y, v.dt_u, v.dt_over_tau_u, v.uw, k, v.n_sub, m0, min(kSubstepBlock, v.n_sub - m0), nullptr,
          nullptr, nullptr, 0);
      break;
    }
    case (int)BatchKernel::Refill:
      refill_block<T, R>(v, v.lat[k & 1], v.grid[cur ^ (L & 1)], v.grid[cur ^ ((L + 1) & 1)], k, it.y);
      break;
    default:  // Force
      force_block<R>(v.grid[cur ^ (L & 1)], v.wall, v.n_wall_edges, v.nnode, v.dk, v.hist, v.flag);
      break;
  }
}

template <class T, class R, int V>
__global__ __launch_bounds__(SubstepVariant<V>::NT) void kb_persistent(const CaseView<T, R> *__restrict__ views,
                                                                       const int4 *__restrict__ items,
                                                                       const BatchPhase *__restrict__ prog,
                                                                       int nphase, int steps) {
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (int s = 0; s < steps; ++s)
    for (int p = 0; p < nphase; ++p) {
      const BatchPhase ph = prog[p];
      for (int i = blockIdx.x; i < ph.n; i += gridDim.x) {
        batch_item<T, R, V>(views, items[ph.first + i], ph.which, ph.m0);
        __syncthreads();  // the next item reuses the LDS
      }
      __threadfence();  // this phase's writes, then every workgroup's, before the next phase reads them
      grid.sync();
      __threadfence();
    }
}

template <class T, class R>
__global__ void k_fill_rest(T *lat, size_t plane, R *grid, int nnode) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < plane)
    for (int q = 0; q < 9; ++q) Stor<T>::st(lat, q * plane + i, q, wgt<R>(q));
  if (i < (size_t)nnode)
    for (int q = 0; q < 9; ++q) grid[(size_t)q * nnode + i] = wgt<R>(q);
}

template <class T>
__global__ void k_to_f64(const T *src, double *dst, size_t plane, size_t nodes) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nodes) return;
  for (int q = 0; q < 9; ++q) dst[q * nodes + i] = (double)Stor<T>::ld(src, q * plane + i, q);
}

// n consecutive elements of one population plane q (storage type E) as FP64
template <class E>
__global__ void k_stage_f64(const E *src, double *dst, size_t n, int q) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)Stor<E>::ld(src, i, q);
}

template <class T>
__global__ void k_from_f64(const double *src, T *dst, size_t plane, size_t nodes) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nodes) return;
  for (int q = 0; q < 9; ++q) {
    const double x = src[q * nodes + i];
    if constexpr (sizeof(T) == 8) Stor<T>::st(dst, q * plane + i, q, x);
    else Stor<T>::st(dst, q * plane + i, q, (float)x);
  }
}

// ---- structured refinement levels ---------------------------------------------
// Interface exchange between a level and the next finer one (refinement ratio
// 2, acoustic scaling, equal viscosity): pre-collision density, velocity and
// f^neq, the latter rescaled by the ratio of tau Delta x of the two levels
// (first-order Chapman-Enskog), written back as post-collision populations.

// coarse node of perimeter index p
__device__ __forceinline__ void perimeter_node(const LevelBox &b, int p, int &x, int &y) {
  const int W = b.x1 - b.x0, H = b.y1 - b.y0;
  if (p <= W) {
    x = b.x0 + p;
    y = b.y0;
  } else if (p <= 2 * W + 1) {
    x = b.x0 + p - (W + 1);
    y = b.y1;
  } else if (p <= 2 * W + H) {
    x = b.x0;
    y = b.y0 + 1 + p - (2 * W + 2);
  } else {
    x = b.x1;
    y = b.y0 + 1 + p - (2 * W + H + 1);
  }
}

// perimeter index of perimeter node (x, y)
__device__ __forceinline__ int perimeter_index(const LevelBox &b, int x, int y) {
  const int W = b.x1 - b.x0, H = b.y1 - b.y0;
  if (y == b.y0) return x - b.x0;
  if (y == b.y1) return W + 1 + x - b.x0;
  if (x == b.x0) return 2 * W + 2 + y - b.y0 - 1;
  return 2 * W + H + 1 + y - b.y0 - 1;
}

template <class T, class R>
__global__ __launch_bounds__(256) void k_box_moments(const T *__restrict__ P, int nx, int ny, size_t plane, int bc,
                                                     LevelBox box, R *__restrict__ m) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x, n = 2 * (box.x1 - box.x0 + box.y1 - box.y0);
  if (p >= n) return;
  int x, y;
  perimeter_node(box, p, x, y);
  R f[9], e[9], rho, ux, uy;
  pull<T, R>(P, nx, ny, plane, bc, x, y, f);
  moments<R>(f, rho, ux, uy);
  equilibrium<R>(rho, ux, uy, e);
  m[p] = rho;
  m[n + p] = ux;
  m[2 * n + p] = uy;
#pragma unroll
  for (int q = 0; q < 9; ++q) m[(3 + q) * n + p] = f[q] - e[q];
}

template <class T, class R>
__global__ __launch_bounds__(256) void k_prolong(const R *__restrict__ m0, const R *__restrict__ m1, LevelBox box,
                                                 R tw1, R kf, T *__restrict__ F, int nxf, int nyf, size_t planef) {
  const LevelBox fb{0, 0, nxf - 1, nyf - 1};
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 2 * (nxf - 1 + nyf - 1)) return;
  int i, j;
  perimeter_node(fb, q, i, j);
  // coarse position (x0 + i/2, y0 + j/2): a perimeter node, or the midpoint
  // of two along the perimeter
  const int X2 = 2 * box.x0 + i, Y2 = 2 * box.y0 + j;
  const int xa = X2 >> 1, ya = Y2 >> 1;
  const int pa = perimeter_index(box, xa, ya), pb = perimeter_index(box, xa + (X2 & 1), ya + (Y2 & 1));
  const int n = 2 * (box.x1 - box.x0 + box.y1 - box.y0);
  const R tw0 = R(1) - tw1, half = R(0.5);
  R g[12];
#pragma unroll
  for (int r = 0; r < 12; ++r)
    g[r] = tw0 * (half * (m0[r * n + pa] + m0[r * n + pb])) + tw1 * (half * (m1[r * n + pa] + m1[r * n + pb]));
  R e[9];
  equilibrium<R>(g[0], g[1], g[2], e);
  const size_t c = (size_t)j * nxf + i;
#pragma unroll
  for (int k = 0; k < 9; ++k) Stor<T>::st(F, k * planef + c, k, e[k] + kf * g[3 + k]);
}

template <class T, class R>
__global__ __launch_bounds__(256) void k_restrict(const T *__restrict__ Fprev, int nxf, int nyf, size_t planef,
                                                  LevelBox box, R kc, T *__restrict__ Cb, int nx, size_t plane) {
  const LevelBox ib{box.x0 + 1, box.y0 + 1, box.x1 - 1, box.y1 - 1};
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= 2 * (ib.x1 - ib.x0 + ib.y1 - ib.y0)) return;
  int x, y;
  perimeter_node(ib, p, x, y);
  R g[9], e[9], rho, ux, uy;
  pull<T, R>(Fprev, nxf, nyf, planef, 3, 2 * (x - box.x0), 2 * (y - box.y0), g);
  moments<R>(g, rho, ux, uy);
  equilibrium<R>(rho, ux, uy, e);
  const size_t c = (size_t)y * nx + x;
#pragma unroll
  for (int q = 0; q < 9; ++q) Stor<T>::st(Cb, q * plane + c, q, e[q] + kc * (g[q] - e[q]));
}

inline unsigned blocks(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

template <class T, class R>
void LevelKernels<T, R>::box_moments(const T *P, int nx, int ny, size_t plane, int bc, LevelBox box, R *m,
                                     hipStream_t s) {
  hipLaunchKernelGGL((k_box_moments<T, R>), dim3(blocks(box.perimeter(), 256)), dim3(256), 0, s, P, nx, ny, plane,
                     bc, box, m);
}

template <class T, class R>
void LevelKernels<T, R>::prolong(const R *m0, const R *m1, LevelBox box, double tw1, double kf, T *F, int nxf,
                                 int nyf, size_t planef, hipStream_t s) {
  hipLaunchKernelGGL((k_prolong<T, R>), dim3(blocks(2 * (nxf - 1 + nyf - 1), 256)), dim3(256), 0, s, m0, m1, box,
                     (R)tw1, (R)kf, F, nxf, nyf, planef);
}

template <class T, class R>
void LevelKernels<T, R>::restrict_level(const T *Fprev, int nxf, int nyf, size_t planef, LevelBox box, double kc,
                                        T *Cb, int nx, size_t plane, hipStream_t s) {
  const int n = 2 * (box.W() - 2 + box.H() - 2);
  hipLaunchKernelGGL((k_restrict<T, R>), dim3(blocks(n, 256)), dim3(256), 0, s, Fprev, nxf, nyf, planef, box,
                     (R)kc, Cb, nx, plane);
}

int substep_block(int variant) {
  switch (variant) {
    case 8: return SubstepVariant<8>::H;
    case 9: return SubstepVariant<9>::H;
    case 10: return SubstepVariant<10>::H;
    default: return kSubstepBlock;
  }
}

void substep_tile(int variant, int *tx, int *ty) {
  switch (variant) {
#define HLBM_TILE(V)                     \
  case V:                                \
    *tx = SubstepVariant<V>::G::TX;      \
    *ty = SubstepVariant<V>::G::TY;      \
    break;
    HLBM_TILE(1) HLBM_TILE(2) HLBM_TILE(3) HLBM_TILE(4) HLBM_TILE(5) HLBM_TILE(6) HLBM_TILE(7)
#undef HLBM_TILE
    default:
      *tx = SubstepVariant<0>::G::TX;
      *ty = SubstepVariant<0>::G::TY;
      break;
  }
}

template <class T, class R>
hipError_t Kernels<T, R>::prepare() {
#define HLBM_LDS(V)                                                                                                  \
  {reinterpret_cast<const void *>(&k_grid_substeps<R, V>), reinterpret_cast<const void *>(&kb_grid_substeps<T, R, V>), \
   (int)substeps_lds_bytes<R, typename SubstepVariant<V>::G,                                                          \
                           substeps_double_buffer<R, typename SubstepVariant<V>::G>()>(),                            \
   (int)substeps_lds_bytes<R, typename SubstepVariant<V>::G>()}
  struct FnLds {
    const void *f, *fb;
    int lds, lds_b;
  };
  const FnLds fns[] = {HLBM_LDS(0), HLBM_LDS(1), HLBM_LDS(2), HLBM_LDS(3),
             HLBM_LDS(4), HLBM_LDS(5), HLBM_LDS(6), HLBM_LDS(7)};
#undef HLBM_LDS
  for (const auto &e : fns) {
    hipError_t rc = hipFuncSetAttribute(e.f, hipFuncAttributeMaxDynamicSharedMemorySize, e.lds);
    if (rc == hipSuccess) rc = hipFuncSetAttribute(e.fb, hipFuncAttributeMaxDynamicSharedMemorySize, e.lds_b);
    if (rc != hipSuccess) return rc;
  }
#define HLBM_LDS1(V)                                                                                      \
  {reinterpret_cast<const void *>(&k_grid_substeps<R, V>), nullptr,                                       \
   (int)substeps_lds_bytes<R, typename SubstepVariant<V>::G,                                              \
                           substeps_double_buffer<R, typename SubstepVariant<V>::G>()>(), 0}
  const FnLds single[] = {HLBM_LDS1(8), HLBM_LDS1(9), HLBM_LDS1(10)};
#undef HLBM_LDS1
  for (const auto &e : single) {
    const hipError_t rc = hipFuncSetAttribute(e.f, hipFuncAttributeMaxDynamicSharedMemorySize, e.lds);
    if (rc != hipSuccess) return rc;
  }
  return hipSuccess;
}

template <class T, class R>
void Kernels<T, R>::fill_rest(T *lat, size_t plane, R *grid, int nnode, hipStream_t s) {
  const size_t n = plane > (size_t)nnode ? plane : (size_t)nnode;
  hipLaunchKernelGGL((k_fill_rest<T, R>), dim3(blocks(n, 256)), dim3(256), 0, s, lat, plane, grid, nnode);
}

// workgroups for the interface donors of a grid in a launch of nt lanes
// (four lanes per node), rounded up to a multiple of the eight XCDs
static int donor_groups(int n_iface, int nt) {
  const int n = (int)blocks((size_t)4 * n_iface, nt);
  return (n + 7) / 8 * 8;
}

template <class T, class R>
void Kernels<T, R>::stream_collide(const CaseView<T, R> &v, hipStream_t s, hipEvent_t start, hipEvent_t stop,
                                   int threads, int rows, int order, bool donors) {
  const int nt = threads > 0 ? threads : kLatticeThreads, rpt = rows > 0 ? rows : kLatticeRows;
  if (v.ww <= 0 || v.wh <= 0) {
    if (donors) interface_donors(v, s);
    return;
  }
  const int nbx = (int)blocks(v.ww, nt), nblocks = nbx * ((v.wh + rpt - 1) / rpt);
  const int ndon = donors && v.n_iface > 0 ? donor_groups(v.n_iface, nt) : 0;
  const dim3 g(nblocks + ndon);
  const int band = order & 1;
#define HLBM_K1(RPT)                                                                                            \
  if (start) /* events taken by the command processor at the kernel's own start and end */                    \
    hipExtLaunchKernelGGL((k_stream_collide<T, R, RPT>), g, dim3(nt), 0, s, start, stop, 0, v, nbx, nblocks,     \
                          band, ndon);                                                                         \
  else                                                                                                         \
    hipLaunchKernelGGL((k_stream_collide<T, R, RPT>), g, dim3(nt), 0, s, v, nbx, nblocks, band, ndon)
  switch (rpt) {
    case 4: HLBM_K1(4); break;
    case 2: HLBM_K1(2); break;
    default: HLBM_K1(1); break;
  }
#undef HLBM_K1
}

template <class T, class R>
void Kernels<T, R>::stream_collide2(const CaseView<T, R> &v, hipStream_t s, hipEvent_t start, hipEvent_t stop,
                                    int order, bool donors) {
  const int tiles_x = (int)blocks(v.nx, kTwoStepTX), tiles = tiles_x * (int)blocks(v.ny, kTwoStepTY);
  // three tile rows and five tiles: measured on 2048^2 against other offsets
  const int segments = order == 1 ? 3 * tiles_x + 5 : -1;
  constexpr int nt = kTwoStepTX * kTwoStepTY;
  const int ndon = donors && v.n_iface > 0 ? donor_groups(v.n_iface, nt) : 0;
  if (start || stop)
    hipExtLaunchKernelGGL((k_stream_collide2<T, R>), dim3(tiles + ndon), dim3(nt), 0, s, start, stop, 0, v, tiles_x,
                          segments, ndon);
  else
    hipLaunchKernelGGL((k_stream_collide2<T, R>), dim3(tiles + ndon), dim3(nt), 0, s, v, tiles_x, segments, ndon);
}

template <class T, class R>
void Kernels<T, R>::lattice_from_grid(const CaseView<T, R> &v, const R *grid, hipStream_t s) {
  hipLaunchKernelGGL((k_lattice_from_grid<T, R>), dim3(blocks(v.k2_w, 256), v.k2_h), dim3(256), 0, s, v, grid);
}

template <class T, class R>
void Kernels<T, R>::interface_donors(const CaseView<T, R> &v, hipStream_t s) {
  hipLaunchKernelGGL((k_interface_donors<T, R>), dim3(blocks((size_t)4 * v.n_iface, 256)), dim3(256), 0, s, v);
}

template <class T, class R>
template <int V>
void Kernels<T, R>::grid_substeps_v(const CaseView<T, R> &v, const R *f, R *fout, int m0, int count, hipStream_t s,
                                    R *tape, R *wtape, const int *widx, int nwall, hipEvent_t start,
                                    hipEvent_t stop) {
  using SV = SubstepVariant<V>;
  const int tiles_x = (v.nux + SV::G::TX - 1) / SV::G::TX, tiles_y = (v.nuy + SV::G::TY - 1) / SV::G::TY;
  constexpr size_t lds = substeps_lds_bytes<R, typename SV::G, substeps_double_buffer<R, typename SV::G>()>();
  if (start || stop)
    hipExtLaunchKernelGGL((k_grid_substeps<R, V>), dim3(tiles_x * tiles_y), dim3(SV::NT), lds, s, start, stop, 0,
                          f, fout,
                          (const R *)v.star_f, (const R *)v.star_n, v.ncode, v.tab, v.nux, v.nuy, tiles_x,
                          tiles_x * tiles_y, v.dt_u, v.dt_over_tau_u, v.uw, (const int64_t *)v.dk, v.n_sub, m0,
                          count, tape, wtape, widx, nwall);
  else
    hipLaunchKernelGGL((k_grid_substeps<R, V>), dim3(tiles_x * tiles_y), dim3(SV::NT), lds, s, f, fout,
                       (const R *)v.star_f,
                       (const R *)v.star_n, v.ncode, v.tab, v.nux, v.nuy, tiles_x, tiles_x * tiles_y, v.dt_u,
                       v.dt_over_tau_u, v.uw, (const int64_t *)v.dk, v.n_sub, m0, count, tape, wtape, widx, nwall);
}

template <class T, class R>
void Kernels<T, R>::grid_substeps(const CaseView<T, R> &v, const R *f, R *fout, int m0, int count, hipStream_t s,
                                  R *tape, R *wtape, const int *widx, int nwall, int variant, hipEvent_t start,
                                  hipEvent_t stop) {
  switch (variant < 0 ? default_substep_variant<R>() : variant) {
#define HLBM_V(V) \
  case V: grid_substeps_v<V>(v, f, fout, m0, count, s, tape, wtape, widx, nwall, start, stop); break;
    HLBM_V(1) HLBM_V(2) HLBM_V(3) HLBM_V(4) HLBM_V(5) HLBM_V(6) HLBM_V(7) HLBM_V(8) HLBM_V(9) HLBM_V(10)
#undef HLBM_V
    default: grid_substeps_v<0>(v, f, fout, m0, count, s, tape, wtape, widx, nwall, start, stop); break;
  }
}

template <class T, class R>
void Kernels<T, R>::refill(const CaseView<T, R> &v, const R *fold, R *fnew, hipStream_t s) {
  hipLaunchKernelGGL((k_refill<T, R>), dim3(blocks(v.nnode, 256)), dim3(256), 0, s, v, fold, fnew);
}

template <class T, class R>
void Kernels<T, R>::mesh_deform(const MeshDeformView<R> &g, hipStream_t s) {
  hipLaunchKernelGGL((k_mesh_deform<R>), dim3(blocks(g.nnode + g.ntri + g.nwall, kDeformThreads)),
                     dim3(kDeformThreads), 0, s, g);
}

template <class T, class R>
void Kernels<T, R>::force(const CaseView<T, R> &v, const R *f, hipStream_t s, int advance) {
  hipLaunchKernelGGL((k_force<R>), dim3(1), dim3(256), 0, s, f, v.wall, v.n_wall_edges, v.nnode, v.dk, v.hist,
                     v.flag, v.mot, const_cast<StepParams *>(v.params), const_cast<R *>(v.uw), v.n_sub, advance);
}

template <class T, class R>
void Kernels<T, R>::refill_force(const CaseView<T, R> &v, const R *fold, R *fnew, unsigned *done, hipStream_t s) {
  hipLaunchKernelGGL((k_refill_force<T, R>), dim3(1 + blocks(v.nnode, 256)), dim3(256), 0, s, v, fold, fnew, done);
}

template <class T, class R>
void Kernels<T, R>::copy_step(const int64_t *from, int64_t *to, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_step, dim3(1), dim3(64), 0, s, from, to);
}

template <class T, class R>
void Kernels<T, R>::advance_step(const CaseView<T, R> &v, hipStream_t s) {
  hipLaunchKernelGGL(k_advance_step, dim3(1), dim3(64), 0, s, v.dk);
}

template <class T, class R>
void Kernels<T, R>::lattice_to_f64(const T *src, double *dst, size_t plane, size_t nodes, hipStream_t s) {
  hipLaunchKernelGGL((k_to_f64<T>), dim3(blocks(nodes, 256)), dim3(256), 0, s, src, dst, plane, nodes);
}

template <class T, class R>
void Kernels<T, R>::lattice_stage_f64(const T *src, double *dst, size_t n, int q, hipStream_t s) {
  hipLaunchKernelGGL((k_stage_f64<T>), dim3(blocks(n, 256)), dim3(256), 0, s, src, dst, n, q);
}

template <class T, class R>
void Kernels<T, R>::grid_stage_f64(const R *src, double *dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_stage_f64<R>), dim3(blocks(n, 256)), dim3(256), 0, s, src, dst, n, 0);
}

template <class T, class R>
void Kernels<T, R>::lattice_from_f64(const double *src, T *dst, size_t plane, size_t nodes, hipStream_t s) {
  hipLaunchKernelGGL((k_from_f64<T>), dim3(blocks(nodes, 256)), dim3(256), 0, s, src, dst, plane, nodes);
}

template <class T, class R>
void Kernels<T, R>::batched(BatchKernel which, const CaseView<T, R> *views, const int4 *items, int nitems, int m0,
                            int threads, hipStream_t s, int rows) {
  if (nitems <= 0) return;
  const dim3 g(nitems);
  switch (which) {
    case BatchKernel::StreamCollide:
      switch (rows) {
        case 4: hipLaunchKernelGGL((kb_stream_collide<T, R, 4>), g, dim3(threads), 0, s, views, items); break;
        case 2: hipLaunchKernelGGL((kb_stream_collide<T, R, 2>), g, dim3(threads), 0, s, views, items); break;
        default: hipLaunchKernelGGL((kb_stream_collide<T, R, 1>), g, dim3(threads), 0, s, views, items); break;
      }
      break;
    case BatchKernel::LatticeFromGrid:
      hipLaunchKernelGGL((kb_lattice_from_grid<T, R>), g, dim3(256), 0, s, views, items);
      break;
    case BatchKernel::InterfaceDonors:
      hipLaunchKernelGGL((kb_interface_donors<T, R>), g, dim3(256), 0, s, views, items);
      break;
    case BatchKernel::GridSubsteps:  // threads: the sub-step variant (-1: default)
      switch (threads < 0 ? default_substep_variant<R>() : threads) {
#define HLBM_KB(V)                                                                                                \
  hipLaunchKernelGGL((kb_grid_substeps<T, R, V>), g, dim3(SubstepVariant<V>::NT),                              \
                     (substeps_lds_bytes<R, typename SubstepVariant<V>::G>()), s, views, items, m0)
        case 1: HLBM_KB(1); break;
        case 2: HLBM_KB(2); break;
        case 3: HLBM_KB(3); break;
        case 4: HLBM_KB(4); break;
        case 5: HLBM_KB(5); break;
        case 6: HLBM_KB(6); break;
        case 7: HLBM_KB(7); break;
        default: HLBM_KB(0); break;
#undef HLBM_KB
      }
      break;
    case BatchKernel::Refill:
      hipLaunchKernelGGL((kb_refill<T, R>), g, dim3(256), 0, s, views, items);
      break;
    case BatchKernel::Force:
      hipLaunchKernelGGL((kb_force<T, R>), g, dim3(256), 0, s, views, items);
      break;
  }
}

template <class T, class R>
void Kernels<T, R>::mesh_substep(const CaseView<T, R> &v, const R *f, R *fout, int m, hipStream_t s,
                                 hipEvent_t start, hipEvent_t stop) {
  const dim3 g(blocks(v.nnode, kMeshThreads));
  if (start || stop)
    hipExtLaunchKernelGGL((k_mesh_substep<T, R>), g, dim3(kMeshThreads), 0, s, start, stop, 0, v, f, fout, m);
  else
    hipLaunchKernelGGL((k_mesh_substep<T, R>), g, dim3(kMeshThreads), 0, s, v, f, fout, m);
}

template <class T, class R>
hipError_t Kernels<T, R>::batched_persistent(const CaseView<T, R> *views, const int4 *items, const BatchPhase *prog,
                                             int nphase, int steps, int variant, int max_groups, hipStream_t s) {
  const void *fn = nullptr;
  int nt = 0, lds = 0;
  switch (variant) {
#define HLBM_P(V)                                                                        \
  case V:                                                                                \
    fn = reinterpret_cast<const void *>(&kb_persistent<T, R, V>);                        \
    nt = SubstepVariant<V>::NT;                                                          \
    lds = (int)substeps_lds_bytes<R, typename SubstepVariant<V>::G>();                   \
    break;
    HLBM_P(4) HLBM_P(5) HLBM_P(6) HLBM_P(7)
#undef HLBM_P
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  int dev = 0, per_cu = 0, cus = 0;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nt, lds);
  if (e != hipSuccess) return e;
  // every workgroup must be resident at once for the grid barrier
  const int groups = std::max(1, std::min(max_groups, per_cu * cus));
  void *args[] = {(void *)&views, (void *)&items, (void *)&prog, (void *)&nphase, (void *)&steps};
  return hipLaunchCooperativeKernel(fn, dim3(groups), dim3(nt), args, lds, s);
}

template <class T, class R>
int Kernels<T, R>::persistent_threads(int variant) {
  switch (variant) {
    case 4: return SubstepVariant<4>::NT;
    case 5: return SubstepVariant<5>::NT;
    case 6: return SubstepVariant<6>::NT;
    case 7: return SubstepVariant<7>::NT;
    default: return 0;
  }
}

template struct Kernels<double, double>;
template struct Kernels<float, float>;
template struct Kernels<__half, float>;
template struct LevelKernels<double, double>;
template struct LevelKernels<float, float>;
template struct LevelKernels<__half, float>;

}  // namespace mghlbm
