// Launch interface of the discrete-adjoint kernels (internal to the library).
//
// The adjoint runs the step of the hybrid method backwards for a cotangent of
// the force history, J = sum_k w_k . F(t_{k+1}), and accumulates dJ/dA,
// dJ/domega and dJ/dtau (tau_s; tau_u = tau_s - 1/2 follows). The discrete
// decisions of the forward run (node status, donor cells, triangles, refill
// types, the number of sub-steps) are held fixed, so J is differentiated
// piece by piece exactly as the forward computed it.
#pragma once

#include "device_common.h"

namespace mghlbm {

// The transposed stencil of a grid node q: slot s holds the coefficients its
// neighbour p (at slot s of q) applies to q, i.e. p's own slot 8 - s; bit s
// of star is set when p reads q's structured-derived value instead of q's f
// (both on the outer ring, Eq.(postcollision2_u)). Nodes with equal
// transposed stencils share one class.
template <class R>
struct AdjClass {
  R Gx[NSLOT];
  R Gy[NSLOT];
  R C[NSLOT];
  int star;
  int type;  // NodeType of q
};

// Everything the adjoint kernels of one reverse step read, by value.
template <class T, class R>
struct AdjCtx {
  // lattice
  int nx, ny, bc, has_grid;
  size_t plane;      // population-plane stride of Lt, Lb_next and Lb
  const T *Lt;       // taped lattice of step k after the grid-to-lattice writes (L'_k)
  const R *Lb_next;  // adjoint of L_{k+1}, [9][ny][nx]
  R *Lb;             // adjoint of L'_k, then of L_k
  // step k
  StepParams P;
  double dyA, dyW;    // d y_k / dA, d y_k / d omega
  double dyA1, dyW1;  // d y_{k+1} / dA, d y_{k+1} / d omega
  double wfx, wfy;    // cotangent of F(t_{k+1})
  // parameters
  double tau, tau_u;
  R inv_tau, g_post, k_neq, dt, dt_tau;
  // grid
  dev::GridGeom gg;
  int nnode, n_iface, n_wall;
  const int *ncode;  // per node: 16 class + 4 zero_diag + type (-1: no class)
  const GridClass<R> *tab;
  const int *iface;
  const int *wall_nodes;    // ids of the wall nodes
  const int *widx;          // per grid node: its index among the wall nodes, -1 otherwise
  const unsigned char *ntype;  // per grid node: NodeType
  const int *acls;          // per grid node: 4 transposed stencil class + the diagonal slot
                            // pairs it lacks (bit 0: slots 2 and 6, bit 1: 0 and 8)
  const AdjClass<R> *atab;
  const double *wall_nrm;   // [2][nnode]: sum over a wall node's edges of (len/2) n
  const R *wt;              // [n][3][n_wall] wall-node moments before the velocity is imposed
  const R *U0;              // grid state U_k
  const R *Un;              // grid state after the n sub-steps of step k
  R *star_f, *star_n;       // structured-derived values of step k (recomputed)
  R *M2;                    // [3][nnode] interpolated (rho, u) at interface nodes
  R *sbf, *sbn;             // adjoints of star_f, star_n
  const R *Ub_next;         // adjoint of U_{k+1}
  R *Ubn;                   // adjoint of the grid after the sub-steps
  R *Z1, *Z2;               // [12][nnode] adjoints of interpolated (rho, u, f^neq):
                            // refill type 1 (Z1) and interface donors (Z2)
  unsigned char *zf;        // per grid node: 1 = type-1 refill this step, 2 = interface
  R *Z3;                    // [12][k2_h][k2_w] same for the lattice nodes set from the grid
  int k2_x0, k2_w, k2_h;
  R *E;                     // [9][eh][ew] adjoint of the pre-collision f at donor lattice nodes
  int ex0, ey0, ew, eh;
  R *Vend;                  // outflow ends (bc 2): [4][9][nx] post-collision adjoints of rows 0, 1,
                            // ny-2, ny-1, gathered into the end rows of Lb afterwards
  double *part;             // parameter partial sums [slots][3] (A, omega, tau)
};

// per-sub-step scalars of one launch of the blocked sub-step adjoint
template <class R>
struct AdjSubScal {
  R uw[4];                  // lamina velocity u_w at the end of the sub-step
  double duwA[4], duwW[4];  // its derivatives in A and omega
};

template <class T, class R>
struct AdjKernels {
  // one launch: recompute f*, f^neq* and the interpolated moments of the
  // interface nodes; refill and force adjoints (Ubn from Ub_next; Z1 and zf,
  // partial sums from slot0 on)
  static void star_refill(const AdjCtx<T, R> &c, int slot0, hipStream_t s);
  // sub-steps m_hi, m_hi-1, ..., m_hi-count+1 backwards (count <= 4): per
  // sub-step the wall-velocity adjoint (lamina velocity of that sub-step and
  // its A, omega derivatives in sc, index m_hi - m), then the transposed
  // stencil; ub -> ub_out; tape0: the step's taped grid states, sub-step m
  // at tape0 + 9 m nnode; first/last: the launch holds m = n-1 / m = 0
  // start, stop (optional): events taken at the launch's own start and end
  static void substeps(const AdjCtx<T, R> &c, const R *tape0, const R *ub, R *ub_out, int m_hi, int count,
                       const AdjSubScal<R> &sc, int first, int last, int slot0, hipStream_t s,
                       hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
  // lattice side: donor gather E, stream-collide adjoint, grid-to-lattice adjoint
  static void donor_gather(const AdjCtx<T, R> &c, int slot0, hipStream_t s);
  static void stream_collide(const AdjCtx<T, R> &c, int slot0, hipStream_t s, hipEvent_t start = nullptr,
                             hipEvent_t stop = nullptr);
  static void from_grid(const AdjCtx<T, R> &c, int slot0, hipStream_t s);
  // grid side of the grid-to-lattice adjoint, added into ub (adjoint of U_k)
  static void from_grid_gather(const AdjCtx<T, R> &c, R *ub, int slot0, hipStream_t s);
  // partial-sum slots each launcher uses
  static int refill_slots(const AdjCtx<T, R> &c);
  static int substep_slots(const AdjCtx<T, R> &c);
  static int donor_gather_slots(const AdjCtx<T, R> &c);
  static int stream_collide_slots(const AdjCtx<T, R> &c);
  static int from_grid_slots(const AdjCtx<T, R> &c);
  static int from_grid_gather_slots(const AdjCtx<T, R> &c);
};

// sums part[0 .. nslots) into out[3] in a fixed order
void adj_reduce(const double *part, int nslots, double *out, hipStream_t s);
void set_step_counter(int64_t *dk, int64_t k, hipStream_t s);

extern template struct AdjKernels<double, double>;
extern template struct AdjKernels<float, float>;
extern template struct AdjKernels<__half, float>;

}  // namespace mghlbm
