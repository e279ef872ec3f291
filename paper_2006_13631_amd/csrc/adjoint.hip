// gfx950 discrete-adjoint kernels of the moving-grid hybrid step.
//
// Reverse of one structured step k (forward order: grid-to-lattice writes,
// lattice stream-collide, interface donors, n grid sub-steps, refill, force):
//
//   star        recompute f*, f^neq* (forward arithmetic) and keep the
//               interpolated moments of every interface node
//   refill      per grid node: adjoint of its own type-1 refill (Z1), then a
//               gather of every refill that read it (type 3 barycentric in
//               its column, type 2 and wall copies) plus the force adjoint
//   substep     per sub-step: wall nodes first pulled back through the
//               imposed lamina velocity (from moments the recompute taped),
//               then per grid node its transposed finite-volume stencil
//               class applied to the 3 x 3 neighbours in LDS; structured-derived
//               adjoints accumulate at interface nodes; the last sub-step
//               turns them into the donor adjoint (Z2)
//   donor gather per lattice node near the grid: the bilinear weights of every
//               interface donor and type-1 refill that read it, folded with
//               its own moments into E = dJ/d f_pre
//   stream_collide  per lattice node: BGK adjoint plus E, pushed to the
//               addresses the forward pull read (a permutation: no atomics)
//   from_grid   per lattice node set from the grid: adjoint of
//               Eq.(postcollision2_s) (Z3); the node's tape value is dead
//   from_grid gather  per grid node: barycentric weights of every such
//               lattice node whose triangle holds it
//
// Every scatter of the forward is a gather here, so each output element is
// written by one thread in a fixed order and the gradient is bitwise
// reproducible. Parameter derivatives (A and omega through the grid
// position y_k = A sin(omega k) and the lamina velocity u_w = A omega
// cos(omega t), tau through 1/tau_s, the Eq.(postcollision2_s) factor, the
// Eq.(continuity_stresses) factor and dt_u / tau_u) are summed per block into
// fixed slots and reduced once at the end.
#include <hip/hip_ext.h>

#include <type_traits>

#include "adjoint.h"

namespace mghlbm {
namespace {

using namespace dev;

constexpr int NT = 256;  // lattice-sized kernels
constexpr int NG = 64;   // grid-sized kernels: one wave per workgroup spreads the few
                         // thousand grid nodes over all compute units

inline unsigned blocks(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

// Adds this block's (a, b, c) to slot[0..2]; all BT threads must call it.
template <int BT>
__device__ __forceinline__ void block_accum3(double a, double b, double c, double *slot) {
  __shared__ double red[3][BT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
    c += __shfl_xor(c, o, 64);
  }
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  const int wave = tid >> 6, lane = tid & 63;
  if (lane == 0) {
    red[0][wave] = a;
    red[1][wave] = b;
    red[2][wave] = c;
  }
  __syncthreads();
  if (tid == 0) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int w = 0; w < BT / 64; ++w) {
      s0 += red[0][w];
      s1 += red[1][w];
      s2 += red[2][w];
    }
    slot[0] += s0;
    slot[1] += s1;
    slot[2] += s2;
  }
}

template <class R>
__device__ __forceinline__ double dot12(const R z[12], R rho, R ux, R uy, const R fneq[9]) {
  double s = (double)z[0] * (double)rho + (double)z[1] * (double)ux + (double)z[2] * (double)uy;
#pragma unroll
  for (int q = 0; q < 9; ++q) s += (double)z[3 + q] * (double)fneq[q];
  return s;
}

// x coordinate of grid column i and y coordinate of grid row j at base yb
// (the same expressions as the forward kernels, graded or uniform)
__device__ __forceinline__ double grid_x(const GridGeom &g, int i) {
  return g.gx ? g.xc + g.gx[i] : g.xc + (double)(i - g.nux / 2) * g.h;
}
__device__ __forceinline__ double grid_y(const GridGeom &g, double yb, int j) {
  return g.gy ? yb + g.gy[j] : yb + ((double)j - 0.5 * (double)(g.nuy - 1)) * g.h;
}
// height of grid cell row cj (rows cj, cj + 1)
__device__ __forceinline__ double cell_height(const GridGeom &g, int cj) {
  return g.gy ? g.gy[cj + 1] - g.gy[cj] : g.h;
}
// first and last of the graded rows (columns) whose local coordinate lies in
// [lo, hi], widened by `pad` on either side and clamped to the grid
__device__ __forceinline__ void graded_span(const double *v, int n, double lo, double hi, int pad, int &first,
                                            int &last) {
  first = max(graded_cell(v, n, lo) - pad, 0);
  last = min(graded_cell(v, n, hi) + 1 + pad, n - 1);
}

// ---- star: f*, f^neq* of step k and the interpolated moments ----------------
template <class T, class R>
__device__ __forceinline__ void adj_star_block(const AdjCtx<T, R> &c, int bx) {
  const int gt = bx * NG + threadIdx.x;
  const int t = gt >> 2, d = gt & 3;
  const bool valid = t < c.n_iface;
  R acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = R(0);
  int p = 0;
  if (valid) {
    p = c.iface[t];
    const int i = p % c.gg.nux, j = p / c.gg.nux;
    donor_corner<T, R>(c.Lt, c.nx, c.ny, c.plane, c.bc, grid_x(c.gg, i), grid_y(c.gg, c.P.ybase, j), d, acc);
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    acc[k] += __shfl_xor(acc[k], 1, 64);
    acc[k] += __shfl_xor(acc[k], 2, 64);
  }
  if (!valid) return;
  R e[9];
  equilibrium<R>(acc[0], acc[1], acc[2], e);
  const size_t N = (size_t)c.nnode;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    if ((q & 3) != d) continue;
    const R n = c.k_neq * acc[3 + q];
    c.star_n[q * N + p] = n;
    c.star_f[q * N + p] = e[q] + n;
  }
  if (d < 3) c.M2[d * N + p] = acc[d];
}

// ---- refill and force adjoint -------------------------------------------------
template <class T, class R>
__device__ __forceinline__ void adj_refill_block(const AdjCtx<T, R> &c, int slot0, int bx) {
  const int q = bx * NG + threadIdx.x;
  const size_t N = (size_t)c.nnode;
  const GridGeom &g = c.gg;
  double pA = 0.0, pW = 0.0, pT = 0.0;
  if (q < c.nnode) {
    const int i = q % g.nux, j = q / g.nux;
    const int tq = c.ncode[q] & 3;
    // (a) this node's own type-1 refill: adjoint of the interpolated moments
    R z[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) z[k] = R(0);
    unsigned char flag = tq == NODE_INTERFACE ? 2 : 0;
    int kind = 0;
    if (tq != NODE_WALL) kind = refill_cell(g, c.P.ybase, c.P.ybase1, i, j).kind;
    R ub[9];
#pragma unroll
    for (int s = 0; s < 9; ++s) ub[s] = c.Ub_next[s * N + q];
    if (kind == 1) {
      R rho, ux, uy, fneq[9];
      lattice_bilinear<T, R>(c.Lt, c.nx, c.ny, c.plane, c.bc, grid_x(g, i), grid_y(g, c.P.ybase1, j), rho, ux,
                             uy, fneq);
      equilibrium_vjp<R>(rho, ux, uy, ub, z[0], z[1], z[2]);
      double sn = 0.0;
#pragma unroll
      for (int s = 0; s < 9; ++s) {
        z[3 + s] = c.k_neq * ub[s];
        sn += (double)ub[s] * (double)fneq[s];
      }
      pT += sn / (2.0 * c.tau * c.tau);  // d(1 - 1/(2 tau))/d tau
      flag |= 1;
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) c.Z1[k * N + q] = z[k];
    c.zf[q] = flag;
    // (b) every refill that read this node of the old grid
    R acc[9];
#pragma unroll
    for (int s = 0; s < 9; ++s) acc[s] = (tq == NODE_WALL || kind == 2) ? ub[s] : R(0);
    R un[9];
#pragma unroll
    for (int s = 0; s < 9; ++s) un[s] = c.Un[s * N + q];
    double dsum = 0.0;
    // a new node jj lands near old row jj + delta; its triangle's rows are
    // within one (two next to the lamina) of that
    int jlo, jhi;
    if (g.gy) {  // graded: new rows whose position lies within old rows j - 2 .. j + 2
      const double dy = c.P.ybase1 - c.P.ybase;
      graded_span(g.gy, g.nuy, g.gy[max(j - 2, 0)] - dy, g.gy[min(j + 2, g.nuy - 1)] - dy, 1, jlo, jhi);
    } else {
      const double delta = (c.P.ybase1 - c.P.ybase) / g.h;
      jlo = max((int)ceil((double)j - 2.0 - delta) - 1, 0);
      jhi = min((int)ceil((double)j + 2.0 - delta), g.nuy - 1);
    }
    for (int jj = jlo; jj <= jhi; ++jj) {
      for (int ii = max(i - 1, 0); ii <= min(i + 1, g.nux - 1); ++ii) {
        const int p = jj * g.nux + ii;
        if ((c.ncode[p] & 3) == NODE_WALL) continue;
        const RefillCell r = refill_cell(g, c.P.ybase, c.P.ybase1, ii, jj);
        if (r.kind != 3) continue;
        int node[3];
        double lam[3], dl[3];
        cell_triangle(r.ci, r.cj, g.nux, r.a, r.b, node, lam, dl, r.tri);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          if (node[a] != q) continue;
          const R l = R(lam[a]);
          double d = 0.0;
#pragma unroll
          for (int s = 0; s < 9; ++s) {
            const R u = c.Ub_next[s * N + p];
            acc[s] += l * u;
            d += (double)u * (double)un[s];
          }
          // graded: the cell coordinate b = (y_{k+1} - y_k + const)/(cell height)
          dsum += g.gy ? dl[a] * d / cell_height(g, r.cj) : dl[a] * d;
        }
      }
    }
    // uniform: the new node's old-grid coordinate t = (y_{k+1} - y_k)/h + const
    const double hs = g.gy ? 1.0 : g.h;
    pA += dsum * (c.dyA1 - c.dyA) / hs;
    pW += dsum * (c.dyW1 - c.dyW) / hs;
    // (c) force on the lamina at t_{k+1}
    if (tq == NODE_WALL) {
      const double nx = c.wall_nrm[q], ny = c.wall_nrm[N + q];
      R rho, ux, uy;
      moments<R>(un, rho, ux, uy);
      R gb[9], fb[9];
#pragma unroll
      for (int s = 0; s < 9; ++s) {
        const double cx = CXd[s], cy = CYd[s];
        gb[s] = R(-(cx * cx * c.wfx * nx + cx * cy * (c.wfx * ny + c.wfy * nx) + cy * cy * c.wfy * ny));
      }
      const R rb = R(-(c.wfx * nx + c.wfy * ny) / 3.0);
      node_chain<R>(rho, ux, uy, rb, R(0), R(0), gb, fb);
#pragma unroll
      for (int s = 0; s < 9; ++s) acc[s] += fb[s];
    }
#pragma unroll
    for (int s = 0; s < 9; ++s) c.Ubn[s * N + q] = acc[s];
  }
  block_accum3<NG>(pA, pW, pT, c.part + 3 * (size_t)(slot0 + bx));
}

// The star recomputation and the refill adjoint share a launch: neither
// reads what the other writes (star: f*, f^neq*, moments of the interface
// nodes from the taped lattice; refill: Z1, zf, Ubn and its partial sums).
template <class T, class R>
__global__ __launch_bounds__(NG) void k_adj_star_refill(AdjCtx<T, R> c, int slot0, int nstar) {
  if ((int)blockIdx.x < nstar) adj_star_block<T, R>(c, blockIdx.x);
  else adj_refill_block<T, R>(c, slot0, (int)blockIdx.x - nstar);
}

// ---- one sub-step backwards -----------------------------------------------------
// Wall nodes: the forward output o of Eq.(ulbe) is mapped to
// W(o) = o + f^eq(rho(o), (0, u_w)) - f^eq(rho(o), u(o)); the adjoint of the
// new state is pulled back through W'(o)^T (which needs only the moments of
// o, taped by the recompute) before the stencil.
template <class R>
__device__ __forceinline__ void wall_vjp(R rho, R ux, R uy, R uw, R u[9], R &d_uw) {
  R ar, axx, ayy, arw, axw, ayw;
  equilibrium_vjp<R>(rho, ux, uy, u, ar, axx, ayy);
  equilibrium_vjp<R>(rho, R(0), uw, u, arw, axw, ayw);
  const R inv = R(1) / rho;
  const R bx = -axx * inv, by = -ayy * inv;
  const R base = arw - ar - bx * ux - by * uy;
#pragma unroll
  for (int q = 0; q < 9; ++q) u[q] = u[q] + base + bx * R(CXd[q]) + by * R(CYd[q]);
  d_uw = ayw;
}

// Transposed Eq.(ulbe)/Eq.(postcollision2_u) stencil, up to kAdjBlock
// sub-steps backwards per launch (temporal blocking, as in the forward). A
// workgroup owns an ATX x ATY tile and stages the adjoint of the tile plus a
// kAdjBlock-node halo (zeros outside the grid) in LDS, wall nodes already
// pulled back through the velocity imposition of the first sub-step it
// reverses. Reversing sub-step m updates the region grown by the number of
// sub-steps still to go in the launch: node q applies its transposed
// stencil class to the nine region values around it and the chain of its
// own non-equilibrium part at the taped state U_m; the new value of a wall
// node is at once pulled back through the imposition of sub-step m - 1.
// Lanes are dealt over each sub-step's rectangle. Parameter partials and
// the running sums of the structured-derived adjoints (interface nodes)
// are taken for the tile's own nodes only.
constexpr int ATX = 16, ATY = 4, kAdjBlock = 4, ANT = 256;

template <class T, class R>
__global__ __launch_bounds__(ANT) void k_adj_substeps(AdjCtx<T, R> c, const R *__restrict__ tape0,
                                                      const R *__restrict__ ub, R *__restrict__ ub_out, int m_hi,
                                                      int count, AdjSubScal<R> sc, int first, int last, int slot0) {
  constexpr int H = kAdjBlock, RX = ATX + 2 * H, RY = ATY + 2 * H, RN = RX * RY;
  constexpr int SPER = (RN + ANT - 1) / ANT;
  constexpr int PER = ((ATX + 2 * (H - 1)) * (ATY + 2 * (H - 1)) + ANT - 1) / ANT;
  __shared__ R sob[RN * 9];              // adjoint of the region's grid state
  __shared__ int scls[RN];               // acls of the node, -1 outside the grid
  __shared__ R acc[ATX * ATY * 18];      // running sums (sf, sn) of the tile's interface nodes
  const GridGeom &g = c.gg;
  const size_t N = (size_t)c.nnode;
  const int tiles_x = (g.nux + ATX - 1) / ATX;
  const int x0 = (blockIdx.x % tiles_x) * ATX - H, y0 = (blockIdx.x / tiles_x) * ATY - H;
  double pA = 0.0, pW = 0.0, pT = 0.0;
  auto own = [&](int rx, int ry) { return rx >= H && rx < H + ATX && ry >= H && ry < H + ATY; };
  // stage: the region's adjoint, walls pulled back through sub-step m_hi's imposition
#pragma unroll
  for (int u = 0; u < SPER; ++u) {
    const int idx = threadIdx.x + u * ANT;
    if (idx >= RN) continue;
    const int rx = idx % RX, ry = idx / RX;
    const int gi = x0 + rx, gj = y0 + ry;
    const bool in = gi >= 0 && gj >= 0 && gi < g.nux && gj < g.nuy;
    const int p = in ? gj * g.nux + gi : 0;
    R v[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) v[q] = in ? ub[q * N + p] : R(0);
    scls[idx] = in ? c.acls[p] : -1;
    if (in && c.ntype[p] == NODE_WALL) {
      const R *wt = c.wt + (size_t)m_hi * 3 * c.n_wall;
      const int w = c.widx[p];
      R d_uw;
      wall_vjp<R>(wt[w], wt[c.n_wall + w], wt[2 * c.n_wall + w], sc.uw[0], v, d_uw);
      if (own(rx, ry)) {
        pA += (double)d_uw * sc.duwA[0];
        pW += (double)d_uw * sc.duwW[0];
      }
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) sob[idx * 9 + q] = v[q];
  }
  for (int jn = threadIdx.x; jn < ATX * ATY; jn += ANT) {
    const int gi = x0 + H + jn % ATX, gj = y0 + H + jn / ATX;
    const bool iface = gi < g.nux && gj < g.nuy && c.ntype[gj * g.nux + gi] == NODE_INTERFACE;
    const size_t p = iface ? (size_t)gj * g.nux + gi : 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      acc[jn * 18 + k] = (iface && !first) ? c.sbf[k * N + p] : R(0);
      acc[jn * 18 + 9 + k] = (iface && !first) ? c.sbn[k * N + p] : R(0);
    }
  }
  __syncthreads();

  for (int sub = 0; sub < count; ++sub) {
    const int m = m_hi - sub;
    const int ex = count - 1 - sub;
    const int W = ATX + 2 * ex, NA = W * (ATY + 2 * ex), o = H - ex;
    const R *Um = tape0 + (size_t)m * 9 * N;
    R out[PER][9];
    int at[PER];
    bool upd[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int j = threadIdx.x + u * ANT;
      const int rx = o + j % W, ry = o + j / W;
      const int ci = j < NA ? ry * RX + rx : 0;
      const int acode = j < NA ? scls[ci] : -1;  // 4 class + zero slot pairs
      at[u] = ci;
      upd[u] = acode >= 0;
#pragma unroll
      for (int k = 0; k < 9; ++k) out[u][k] = R(0);
      // a wave whose nodes all lack the same two diagonal neighbours skips
      // those slots (zero weights: the sums are the same)
      const int zl = acode >= 0 ? acode & 3 : 3;
      const int zd = __ballot(!(zl & 1)) == 0 ? 1 : (__ballot(!(zl & 2)) == 0 ? 2 : 0);
      if (!upd[u]) continue;
      const size_t q = (size_t)(y0 + ry) * g.nux + (x0 + rx);
      R f[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) f[k] = Um[k * N + q];
      const AdjClass<R> &cl = c.atab[acode >> 2];
      const int tq = cl.type, star = cl.star;
      R accF[9], accN[9], sf[9], sn[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) accF[k] = accN[k] = sf[k] = sn[k] = R(0);
      auto gather = [&](auto mask) {
        constexpr int M = decltype(mask)::value;
#pragma unroll
      for (int s = 0; s < NSLOT; ++s) {
        if (!((M >> s) & 1)) continue;
        const int ri = ci + (s / 3 - 1) * RX + (s % 3 - 1);
        const R gx = cl.Gx[s], gy = cl.Gy[s], cc = cl.C[s];
        const bool st_s = (star >> s) & 1;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          const R ov = sob[ri * 9 + k];
          const R st = c.dt * (R(CXd[k]) * gx + R(CYd[k]) * gy) * ov;
          const R ct = -c.dt_tau * cc * ov;
          if (st_s) {
            sf[k] += st;
            sn[k] += ct;
          } else {
            accF[k] += st;
            accN[k] += ct;
          }
        }
      }
      };
      if (zd == 1)
        gather(std::integral_constant<int, 0x1FF & ~(1 << 2 | 1 << 6)>{});
      else if (zd == 2)
        gather(std::integral_constant<int, 0x1FF & ~(1 << 0 | 1 << 8)>{});
      else
        gather(std::integral_constant<int, 0x1FF>{});
      // the node's own value: its f, or f* at an interface node
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        if (tq == NODE_INTERFACE) sf[k] += sob[ci * 9 + k];
        else accF[k] += sob[ci * 9 + k];
      }
      R e[9], rho, ux, uy, fb[9];
      moments<R>(f, rho, ux, uy);
      equilibrium<R>(rho, ux, uy, e);
      node_chain<R>(rho, ux, uy, R(0), R(0), R(0), accN, fb);
      double dn = 0.0;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        out[u][k] = accF[k] + fb[k];
        dn += (double)accN[k] * (double)(f[k] - e[k]);
      }
      if (tq == NODE_INTERFACE) {
        double ds = 0.0;
#pragma unroll
        for (int k = 0; k < 9; ++k) ds += (double)sn[k] * (double)c.star_n[k * N + q];
        dn += ds;
      }
      if (own(rx, ry)) {
        // d(dt_u/tau_u)/d tau = -dt_u/tau_u^2: the collision adjoints carry -dt_u/tau_u
        pT += dn * (-1.0 / c.tau_u);
        if (tq == NODE_INTERFACE) {
          const int jn = (ry - H) * ATX + (rx - H);
#pragma unroll
          for (int k = 0; k < 9; ++k) {
            acc[jn * 18 + k] += sf[k];
            acc[jn * 18 + 9 + k] += sn[k];
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      if (!upd[u]) continue;
      const int ci = at[u];
      if (sub + 1 < count) {  // pull a wall node back through sub-step m - 1's imposition
        const int rx = ci % RX, ry = ci / RX;
        const size_t p = (size_t)(y0 + ry) * g.nux + (x0 + rx);
        if (c.ntype[p] == NODE_WALL) {
          const R *wt = c.wt + (size_t)(m - 1) * 3 * c.n_wall;
          const int w = c.widx[p];
          R d_uw;
          wall_vjp<R>(wt[w], wt[c.n_wall + w], wt[2 * c.n_wall + w], sc.uw[sub + 1], out[u], d_uw);
          if (own(rx, ry)) {
            pA += (double)d_uw * sc.duwA[sub + 1];
            pW += (double)d_uw * sc.duwW[sub + 1];
          }
        }
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) sob[ci * 9 + k] = out[u][k];
    }
    __syncthreads();
  }

  // the tile is exact: write it back, with the running star sums
  for (int jn = threadIdx.x; jn < ATX * ATY; jn += ANT) {
    const int rx = H + jn % ATX, ry = H + jn / ATX;
    const int gi = x0 + rx, gj = y0 + ry;
    if (gi >= g.nux || gj >= g.nuy) continue;
    const int ci = ry * RX + rx;
    const size_t q = (size_t)gj * g.nux + gi;
#pragma unroll
    for (int k = 0; k < 9; ++k) ub_out[k * N + q] = sob[ci * 9 + k];
    if (c.ntype[q] != NODE_INTERFACE) continue;
    R sf[9], sn[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      sf[k] = acc[jn * 18 + k];
      sn[k] = acc[jn * 18 + 9 + k];
      c.sbf[k * N + q] = sf[k];
      c.sbn[k * N + q] = sn[k];
    }
    if (last) {
      // donor adjoint: f* = f^eq(rho, u) + k f^neq, f^neq* = k f^neq
      R z[12], tot[9];
      double dk = 0.0;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        tot[k] = sf[k] + sn[k];
        dk += (double)tot[k] * (double)c.star_n[k * N + q];
      }
      equilibrium_vjp<R>(c.M2[q], c.M2[N + q], c.M2[2 * N + q], sf, z[0], z[1], z[2]);
#pragma unroll
      for (int k = 0; k < 9; ++k) z[3 + k] = c.k_neq * tot[k];
#pragma unroll
      for (int k = 0; k < 12; ++k) c.Z2[k * N + q] = z[k];
      // d f^neq*/d tau = (d k/d tau) f^neq = (d k/d tau)/k f^neq*
      pT += dk * (1.0 / (2.0 * c.tau * c.tau)) / (double)c.k_neq;
    }
  }
  block_accum3<ANT>(pA, pW, pT, c.part + 3 * (size_t)(slot0 + blockIdx.x));
}

// ---- donor gather: dJ/d f_pre at lattice nodes read by bilinear donors ------------
template <class T, class R>
__global__ __launch_bounds__(NG) void k_adj_donor_gather(AdjCtx<T, R> c, int slot0) {
  const int x = c.ex0 + blockIdx.x * NG + threadIdx.x;
  const int y = c.ey0 + blockIdx.y;
  const GridGeom &g = c.gg;
  const size_t N = (size_t)c.nnode;
  double pA = 0.0, pW = 0.0;
  if (x < c.ex0 + c.ew) {
    R Eo[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Eo[k] = R(0);
    const bool inside = x >= c.P.ix0 && x <= c.P.ix1 && y >= c.P.iy0 && y <= c.P.iy1;
    if (!inside) {  // donors are discretization nodes
      R zs[12], zA[12], zW[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) zs[k] = zA[k] = zW[k] = R(0);
      bool any = false;
      int ilo, ihi;
      if (g.gx) {
        graded_span(g.gx, g.nux, (double)x - 1.0 - g.xc, (double)x + 1.0 - g.xc, 1, ilo, ihi);
      } else {
        ilo = max(0, (int)floor(((double)x - 1.0 - g.xc) / g.h) + g.nux / 2 - 1);
        ihi = min(g.nux - 1, (int)ceil(((double)x + 1.0 - g.xc) / g.h) + g.nux / 2 + 1);
      }
      for (int i = ilo; i <= ihi; ++i) {
        const double X = grid_x(g, i);
        const int fx = (int)floor(X);
        if (fx != x && fx + 1 != x) continue;
        for (int pos = 0; pos < 2; ++pos) {  // 0: interface donors at y_k, 1: type-1 refill at y_{k+1}
          const double yb = pos ? c.P.ybase1 : c.P.ybase;
          const double dyA = pos ? c.dyA1 : c.dyA, dyW = pos ? c.dyW1 : c.dyW;
          int jlo, jhi;
          if (g.gy) {
            graded_span(g.gy, g.nuy, (double)y - 1.0 - yb, (double)y + 1.0 - yb, 1, jlo, jhi);
          } else {
            const double j0 = ((double)y - yb) / g.h + 0.5 * (double)(g.nuy - 1);
            jlo = max(0, (int)floor(j0 - 1.0 / g.h) - 1);
            jhi = min(g.nuy - 1, (int)ceil(j0 + 1.0 / g.h) + 1);
          }
          const unsigned char need = pos ? 1 : 2;
          const R *Z = pos ? c.Z1 : c.Z2;
          for (int j = jlo; j <= jhi; ++j) {
            const int p = j * g.nux + i;
            if (!(c.zf[p] & need)) continue;
            const double Y = grid_y(g, yb, j);
            const int fy = (int)floor(Y);
            if (fy != y && fy + 1 != y) continue;
            int xd, yd;
            double w, dw;
            bilinear_corner(X, Y, (x - fx) + 2 * (y - fy), xd, yd, w, dw);
            const R wr = R(w), wa = R(dw * dyA), ww = R(dw * dyW);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
              const R z = Z[k * N + p];
              zs[k] += wr * z;
              zA[k] += wa * z;
              zW[k] += ww * z;
            }
            any = true;
          }
        }
      }
      if (any) {
        R f[9], e[9], rho, ux, uy, fneq[9];
        pull<T, R>(c.Lt, c.nx, c.ny, c.plane, c.bc, x, y, f);
        moments<R>(f, rho, ux, uy);
        equilibrium<R>(rho, ux, uy, e);
#pragma unroll
        for (int k = 0; k < 9; ++k) fneq[k] = f[k] - e[k];
        node_chain<R>(rho, ux, uy, zs[0], zs[1], zs[2], zs + 3, Eo);
        pA += dot12<R>(zA, rho, ux, uy, fneq);
        pW += dot12<R>(zW, rho, ux, uy, fneq);
      }
    }
    const size_t plane = (size_t)c.ew * c.eh, at = (size_t)(y - c.ey0) * c.ew + (x - c.ex0);
#pragma unroll
    for (int k = 0; k < 9; ++k) c.E[k * plane + at] = Eo[k];
  }
  block_accum3<NG>(pA, pW, 0.0, c.part + 3 * (size_t)(slot0 + blockIdx.y * gridDim.x + blockIdx.x));
}

// ---- lattice stream-collide adjoint ---------------------------------------------
// Forward at a discretization node: f_post = f - (f - f^eq(f))/tau, f pulled
// from L'_k. Backward: v = (1 - 1/tau) l + (1/tau) (d f^eq/d f)^T l + E, then
// v_q is stored at the address the forward pull read f_q from. Inside the
// fictitious rectangle the forward copied the value, and the copy is never
// read again (such nodes are overwritten from the grid before any
// discretization node reads them), so zeros are pushed.
template <class T, class R>
__global__ __launch_bounds__(NT) void k_adj_stream_collide(AdjCtx<T, R> c, int slot0) {
  const int x = blockIdx.x * NT + threadIdx.x;
  const int y = blockIdx.y;
  double pT = 0.0;
  if (x < c.nx) {
    const size_t plane = c.plane, cc = (size_t)y * c.nx + x;
    size_t idx[9];
    pull_index(c.nx, c.ny, c.plane, c.bc, x, y, idx);
    const bool inside = c.has_grid && x >= c.P.ix0 && x <= c.P.ix1 && y >= c.P.iy0 && y <= c.P.iy1;
    R v[9];
    if (inside) {
#pragma unroll
      for (int q = 0; q < 9; ++q) v[q] = R(0);
    } else {
      R f[9], e[9], l[9], rho, ux, uy;
#pragma unroll
      for (int q = 0; q < 9; ++q) f[q] = Stor<T>::ld(c.Lt, idx[q], q);
#pragma unroll
      for (int q = 0; q < 9; ++q) l[q] = c.Lb_next[q * plane + cc];
      moments<R>(f, rho, ux, uy);
      equilibrium<R>(rho, ux, uy, e);
      R ar, ax, ay;
      equilibrium_vjp<R>(rho, ux, uy, l, ar, ax, ay);
      const R inv = R(1) / rho;
      const R bx = ax * inv, by = ay * inv, base = ar - bx * ux - by * uy;
      double dt = 0.0;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        v[q] = (R(1) - c.inv_tau) * l[q] + c.inv_tau * (base + bx * R(CXd[q]) + by * R(CYd[q]));
        dt += (double)l[q] * (double)(f[q] - e[q]);
      }
      pT += dt / (c.tau * c.tau);
      if (c.has_grid && x >= c.ex0 && x < c.ex0 + c.ew && y >= c.ey0 && y < c.ey0 + c.eh) {
        const size_t eplane = (size_t)c.ew * c.eh, at = (size_t)(y - c.ey0) * c.ew + (x - c.ex0);
#pragma unroll
        for (int q = 0; q < 9; ++q) v[q] += c.E[q * eplane + at];
      }
    }
    if (c.bc == 2) {
      // outflow ends: a source in an end row may have two readers (the next
      // row in, and the end node through the zero-gradient copy) or none;
      // those rows are gathered by k_adj_outflow_ends from the adjoints kept
      // here for the two rows at each end
      const int er = y <= 1 ? y : (y >= c.ny - 2 ? 4 - (c.ny - y) : -1);
      if (er >= 0) {
#pragma unroll
        for (int q = 0; q < 9; ++q) c.Vend[((size_t)er * 9 + q) * c.nx + x] = v[q];
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const size_t row = (idx[q] % plane) / (size_t)c.nx;
        if (row != 0 && row != (size_t)(c.ny - 1)) c.Lb[idx[q]] = v[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 9; ++q) c.Lb[idx[q]] = v[q];
    }
  }
  block_accum3<NT>(0.0, 0.0, pT, c.part + 3 * (size_t)(slot0 + blockIdx.y * gridDim.x + blockIdx.x));
}

// Outflow ends (bc 2): every population of the two end rows of Lb is the sum
// of the adjoints of all (node, population) pairs whose pull read it, found
// among the nine nodes around it, in a fixed order.
template <class T, class R>
__global__ __launch_bounds__(NT) void k_adj_outflow_ends(AdjCtx<T, R> c) {
  const int x = blockIdx.x * NT + threadIdx.x;
  const int end = blockIdx.y;  // 0: row 0, 1: row ny - 1
  if (x >= c.nx) return;
  const int y = end ? c.ny - 1 : 0;
  const size_t plane = c.plane, s = (size_t)y * c.nx + x;
  R acc[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) acc[q] = R(0);
  for (int dy = -1; dy <= 1; ++dy) {
    const int ty = y + dy;
    if (ty < 0 || ty >= c.ny) continue;
    const int er = ty <= 1 ? ty : 4 - (c.ny - ty);  // ty is within two rows of this end
    for (int dx = -1; dx <= 1; ++dx) {
      const int tx = x + dx;
      if (tx < 0 || tx >= c.nx) continue;
      size_t idx[9];
      pull_index(c.nx, c.ny, plane, c.bc, tx, ty, idx);
#pragma unroll
      for (int qp = 0; qp < 9; ++qp) {
        if (idx[qp] % plane != s) continue;
        const int q = (int)(idx[qp] / plane);
        const R v = c.Vend[((size_t)er * 9 + qp) * c.nx + tx];
#pragma unroll
        for (int k = 0; k < 9; ++k)
          if (k == q) acc[k] += v;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) c.Lb[q * plane + s] = acc[q];
}

// ---- grid-to-lattice adjoint, lattice side ---------------------------------------
// Forward: L'(x) = f^eq(rho, u) + g f^neq with barycentric (rho, u, f^neq) from
// the grid at t_k, g = 2 (tau - 1)/(2 tau - 1). Z3 holds the adjoint of the
// interpolated (rho, u, f^neq); the node's incoming adjoint is consumed.
template <class T, class R>
__global__ __launch_bounds__(NT) void k_adj_from_grid(AdjCtx<T, R> c, int slot0) {
  const int x = c.k2_x0 + blockIdx.x * NT + threadIdx.x;
  const int ybot = min(c.P.iy0, c.P.piy0);
  const int y = ybot + (int)blockIdx.y;
  double pT = 0.0;
  if (x < c.k2_x0 + c.k2_w) {
    R z[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) z[k] = R(0);
    if (y <= max(c.P.iy1, c.P.piy1) && from_grid_target(c.P, x, y)) {
      int ci, cj, tri, node[3];
      double a, b, lam[3], dl[3];
      lattice_node_cell(c.gg, c.P.ybase, x, y, ci, cj, a, b, tri);
      cell_triangle(ci, cj, c.gg.nux, a, b, node, lam, dl, tri);
      R rho, ux, uy, fneq[9];
      grid_barycentric<R>(c.U0, c.nnode, node, lam, rho, ux, uy, fneq);
      const size_t plane = c.plane, cc = (size_t)y * c.nx + x;
      R lb[9];
      double dg = 0.0;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        lb[q] = c.Lb[q * plane + cc];
        c.Lb[q * plane + cc] = R(0);
        z[3 + q] = c.g_post * lb[q];
        dg += (double)lb[q] * (double)fneq[q];
      }
      equilibrium_vjp<R>(rho, ux, uy, lb, z[0], z[1], z[2]);
      const double tm = 2.0 * c.tau - 1.0;
      pT += dg * 2.0 / (tm * tm);  // d g / d tau
    }
    const size_t zp = (size_t)c.k2_w * c.k2_h, at = (size_t)blockIdx.y * c.k2_w + (x - c.k2_x0);
#pragma unroll
    for (int k = 0; k < 12; ++k) c.Z3[k * zp + at] = z[k];
  }
  block_accum3<NT>(0.0, 0.0, pT, c.part + 3 * (size_t)(slot0 + blockIdx.y * gridDim.x + blockIdx.x));
}

// ---- grid-to-lattice adjoint, grid side -------------------------------------------
template <class T, class R>
__global__ __launch_bounds__(NG) void k_adj_from_grid_gather(AdjCtx<T, R> c, R *__restrict__ ub, int slot0) {
  const int q = blockIdx.x * NG + threadIdx.x;
  const GridGeom &g = c.gg;
  const size_t N = (size_t)c.nnode;
  double pA = 0.0, pW = 0.0;
  if (q < c.nnode) {
    const int i = q % g.nux, j = q / g.nux;
    const int ybot = min(c.P.iy0, c.P.piy0), ytop = min(max(c.P.iy1, c.P.piy1), ybot + c.k2_h - 1);
    // lattice nodes in the cells around the node: between its neighbouring
    // columns and rows, one lattice node wider
    double xa, xb, ya, yb;
    if (g.gx) {
      xa = grid_x(g, max(i - 1, 0));
      xb = grid_x(g, min(i + 1, g.nux - 1));
      ya = grid_y(g, c.P.ybase, max(j - 1, 0));
      yb = grid_y(g, c.P.ybase, min(j + 1, g.nuy - 1));
    } else {
      const double X0 = grid_x(g, 0), Y0 = grid_y(g, c.P.ybase, 0);
      xa = X0 + (double)(i - 1) * g.h;
      xb = X0 + (double)(i + 1) * g.h;
      ya = Y0 + (double)(j - 1) * g.h;
      yb = Y0 + (double)(j + 1) * g.h;
    }
    const int xlo = max((int)floor(xa) - 1, c.k2_x0);
    const int xhi = min((int)ceil(xb) + 1, c.k2_x0 + c.k2_w - 1);
    const int ylo = max((int)floor(ya) - 1, ybot);
    const int yhi = min((int)ceil(yb) + 1, ytop);
    R zs[12], zd[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) zs[k] = zd[k] = R(0);
    bool any = false;
    const size_t zp = (size_t)c.k2_w * c.k2_h;
    // no candidate can be set from the grid when all of them lie strictly
    // inside the rectangle (not on its edge) or outside both rectangles
    const StepParams &P = c.P;
    const bool deep = xlo > P.ix0 && xhi < P.ix1 && ylo > P.iy0 && yhi < P.iy1;
    const bool away = xhi < min(P.ix0, P.pix0) || xlo > max(P.ix1, P.pix1) || yhi < min(P.iy0, P.piy0) ||
                      ylo > max(P.iy1, P.piy1);
    for (int yl = (deep || away) ? yhi + 1 : ylo; yl <= yhi; ++yl) {
      for (int xl = xlo; xl <= xhi; ++xl) {
        if (!from_grid_target(c.P, xl, yl)) continue;
        int ci, cj, tri, node[3];
        double a, b, lam[3], dl[3];
        lattice_node_cell(g, c.P.ybase, xl, yl, ci, cj, a, b, tri);
        cell_triangle(ci, cj, g.nux, a, b, node, lam, dl, tri);
        const size_t at = (size_t)(yl - ybot) * c.k2_w + (xl - c.k2_x0);
#pragma unroll
        for (int n = 0; n < 3; ++n) {
          if (node[n] != q) continue;
          // graded: d b/d y_k = -1/(cell height) per cell (uniform: -1/h, below)
          const R l = R(lam[n]), d = R(g.gy ? dl[n] / cell_height(g, cj) : dl[n]);
#pragma unroll
          for (int k = 0; k < 12; ++k) {
            const R z = c.Z3[k * zp + at];
            zs[k] += l * z;
            zd[k] += d * z;
          }
          any = true;
        }
      }
    }
    if (any) {
      R f[9], e[9], rho, ux, uy, fneq[9], fb[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) f[k] = c.U0[k * N + q];
      moments<R>(f, rho, ux, uy);
      equilibrium<R>(rho, ux, uy, e);
#pragma unroll
      for (int k = 0; k < 9; ++k) fneq[k] = f[k] - e[k];
      node_chain<R>(rho, ux, uy, zs[0], zs[1], zs[2], zs + 3, fb);
#pragma unroll
      for (int k = 0; k < 9; ++k) ub[k * N + q] += fb[k];
      // uniform: the lattice node's grid coordinate t = (y - y_k)/h + const
      const double dsum = dot12<R>(zd, rho, ux, uy, fneq);
      const double hs = g.gy ? 1.0 : g.h;
      pA += dsum * (-c.dyA / hs);
      pW += dsum * (-c.dyW / hs);
    }
  }
  block_accum3<NG>(pA, pW, 0.0, c.part + 3 * (size_t)(slot0 + blockIdx.x));
}

__global__ __launch_bounds__(NT) void k_adj_reduce(const double *__restrict__ part, int nslots, double *out) {
  __shared__ double red[3][NT];
  double s[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nslots; i += NT)
    for (int k = 0; k < 3; ++k) s[k] += part[3 * (size_t)i + k];
  for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < 3; ++k) {
      double t = 0.0;
      for (int i = 0; i < NT; ++i) t += red[k][i];
      out[k] = t;
    }
  }
}

__global__ void k_set_counter(int64_t *dk, int64_t k) { *dk = k; }

}  // namespace

template <class T, class R>
void AdjKernels<T, R>::star_refill(const AdjCtx<T, R> &c, int slot0, hipStream_t s) {
  const int nstar = (int)blocks((size_t)4 * c.n_iface, NG);
  hipLaunchKernelGGL((k_adj_star_refill<T, R>), dim3(nstar + refill_slots(c)), dim3(NG), 0, s, c, slot0, nstar);
}

template <class T, class R>
int AdjKernels<T, R>::refill_slots(const AdjCtx<T, R> &c) {
  return (int)blocks(c.nnode, NG);
}

template <class T, class R>
int AdjKernels<T, R>::substep_slots(const AdjCtx<T, R> &c) {
  return ((c.gg.nux + ATX - 1) / ATX) * ((c.gg.nuy + ATY - 1) / ATY);
}
template <class T, class R>
void AdjKernels<T, R>::substeps(const AdjCtx<T, R> &c, const R *tape0, const R *ub, R *ub_out, int m_hi, int count,
                                const AdjSubScal<R> &sc, int first, int last, int slot0, hipStream_t s,
                                hipEvent_t start, hipEvent_t stop) {
  if (start || stop)
    hipExtLaunchKernelGGL((k_adj_substeps<T, R>), dim3(substep_slots(c)), dim3(ANT), 0, s, start, stop, 0, c, tape0,
                          ub, ub_out, m_hi, count, sc, first, last, slot0);
  else
    hipLaunchKernelGGL((k_adj_substeps<T, R>), dim3(substep_slots(c)), dim3(ANT), 0, s, c, tape0, ub, ub_out, m_hi,
                       count, sc, first, last, slot0);
}

template <class T, class R>
int AdjKernels<T, R>::donor_gather_slots(const AdjCtx<T, R> &c) {
  return (int)blocks(c.ew, NG) * c.eh;
}
template <class T, class R>
void AdjKernels<T, R>::donor_gather(const AdjCtx<T, R> &c, int slot0, hipStream_t s) {
  hipLaunchKernelGGL((k_adj_donor_gather<T, R>), dim3(blocks(c.ew, NG), c.eh), dim3(NG), 0, s, c, slot0);
}

template <class T, class R>
int AdjKernels<T, R>::stream_collide_slots(const AdjCtx<T, R> &c) {
  return (int)blocks(c.nx, NT) * c.ny;
}
template <class T, class R>
void AdjKernels<T, R>::stream_collide(const AdjCtx<T, R> &c, int slot0, hipStream_t s, hipEvent_t start,
                                      hipEvent_t stop) {
  if (start) {
    hipExtLaunchKernelGGL((k_adj_stream_collide<T, R>), dim3(blocks(c.nx, NT), c.ny), dim3(NT), 0, s, start, stop, 0,
                          c, slot0);
  } else {
    hipLaunchKernelGGL((k_adj_stream_collide<T, R>), dim3(blocks(c.nx, NT), c.ny), dim3(NT), 0, s, c, slot0);
  }
  if (c.bc == 2) hipLaunchKernelGGL((k_adj_outflow_ends<T, R>), dim3(blocks(c.nx, NT), 2), dim3(NT), 0, s, c);
}

template <class T, class R>
int AdjKernels<T, R>::from_grid_slots(const AdjCtx<T, R> &c) {
  return (int)blocks(c.k2_w, NT) * c.k2_h;
}
template <class T, class R>
void AdjKernels<T, R>::from_grid(const AdjCtx<T, R> &c, int slot0, hipStream_t s) {
  hipLaunchKernelGGL((k_adj_from_grid<T, R>), dim3(blocks(c.k2_w, NT), c.k2_h), dim3(NT), 0, s, c, slot0);
}

template <class T, class R>
int AdjKernels<T, R>::from_grid_gather_slots(const AdjCtx<T, R> &c) {
  return (int)blocks(c.nnode, NG);
}
template <class T, class R>
void AdjKernels<T, R>::from_grid_gather(const AdjCtx<T, R> &c, R *ub, int slot0, hipStream_t s) {
  hipLaunchKernelGGL((k_adj_from_grid_gather<T, R>), dim3(from_grid_gather_slots(c)), dim3(NG), 0, s, c, ub, slot0);
}

void adj_reduce(const double *part, int nslots, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(NT), 0, s, part, nslots, out);
}

void set_step_counter(int64_t *dk, int64_t k, hipStream_t s) {
  hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, s, dk, k);
}

template struct AdjKernels<double, double>;
template struct AdjKernels<float, float>;
template struct AdjKernels<__half, float>;

}  // namespace mghlbm
