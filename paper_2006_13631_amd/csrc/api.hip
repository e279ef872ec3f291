// Host runtime and C ABI of the gfx950 HLBM library (see include/hlbm.h).
//
// One case owns: two lattice buffers (ping-pong), two grid buffers, the
// structured-derived interface values, the stencil classes of the grid, a
// per-step table of FP64 scalars computed here (motion, fictitious-rectangle
// bounds, wall velocity at each sub-step) and the force history. A step runs
// the lattice update and the grid path on two HIP streams of default
// priority: within a step the grid path reads only the lattice buffer of
// t_k, which the lattice kernel only reads, so the two proceed concurrently.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "adjoint.h"
#include "hlbm.h"
#include "kernels.h"

// Staging buffer of hlbm_get_state_noalloc: one per GPU, held from module
// load until the process ends. Host code must not use its name as an address
// (it is a host-side stand-in); scratch_on() looks up the device address.
static __device__ __align__(256) double scratch[(size_t)HLBM_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace mghlbm {
namespace {

constexpr size_t kScratchElems = (size_t)HLBM_NOALLOC_SCRATCH_BYTES / sizeof(double);
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, taken once per device with that
// device current (each GPU holds its own copy at its own address).
hipError_t scratch_on(int dev, double **out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = (double *)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Nine population planes of `per` values each (plane q at element q * stride
// of the device array) to the packed FP64 host array out[9][per]: launch(q,
// a, n, buf) converts values a .. a+n-1 of plane q into buf (at most `cap`
// doubles), which is then copied out; the pieces follow each other on
// stream s, so a conversion never overwrites a piece still being copied.
template <class Launch>
hipError_t stage_planes(double *out, size_t per, double *buf, size_t cap, hipStream_t s, Launch launch) {
  for (int q = 0; q < 9; ++q)
    for (size_t a = 0; a < per; a += cap) {
      const size_t n = std::min(cap, per - a);
      launch(q, a, n, buf);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess)
        e = hipMemcpyAsync(out + (size_t)q * per + a, buf, n * sizeof(double), hipMemcpyDeviceToHost, s);
      if (e != hipSuccess) return e;
    }
  return hipStreamSynchronize(s);
}

std::string g_create_error;

constexpr double kMargin = 2.0;  // inset of the fictitious rectangle (lattice units)
constexpr int kGraphSteps = 8;   // structured steps per captured HIP graph (even)

struct Derived {
  double nu, tau_u, A, omega, xc, yc;
  int n;
};

// Derived quantities (Sec. Problem statement; viscosity matching of Sec. 3).
// mesh: the case has an unstructured grid (nux, nuy unused)
Derived derive(const hlbm_config &c, bool mesh = false) {
  Derived d;
  d.nu = (c.tau - 0.5) / 3.0;
  d.tau_u = c.tau - 0.5;
  const bool has_grid = c.nux > 0 || c.nuy > 0 || mesh;
  if (has_grid && c.b > 0.0) {
    d.A = c.kc * c.b / (2.0 * M_PI);
    d.omega = 2.0 * M_PI * d.nu * c.beta / (c.b * c.b);
  } else {
    d.A = 0.0;
    d.omega = 0.0;
  }
  if (c.n_sub > 0) {
    d.n = c.n_sub;
  } else {
    const int n = (int)std::ceil(1.0 / d.tau_u - 1e-9);
    d.n = n < 2 ? 2 : n;
  }
  d.xc = (double)(c.nx / 2);
  d.yc = 0.5 * (double)(c.ny - 1);
  return d;
}

class CaseBase {
 public:
  virtual ~CaseBase() = default;
  virtual int step(int64_t n) = 0;
  // enqueue n steps and return without waiting for them (single cases;
  // other handles step as hlbm_step does)
  virtual int step_async(int64_t n) { return step(n); }
  // wait for the enqueued steps; their status as step() reports it
  virtual int sync() { return 0; }
  // wait for the enqueued steps before another call reads or writes the
  // state (their status stays on the device flag for the next step or sync)
  virtual void drain() {}
  virtual int get_state(int which, void *buf, size_t bytes) = 0;
  virtual int set_state(int which, const void *buf, size_t bytes) = 0;
  // get_state of the lattice and grid states through the static staging
  // buffer, without allocating
  virtual int get_state_noalloc(int which, void *buf, size_t bytes) {
    (void)which;
    (void)buf;
    (void)bytes;
    err = "this handle has no allocation-free state read";
    return HLBM_E_UNSUPPORTED;
  }
  virtual int force(double *hist, int64_t cap, int64_t *n_out, double t0, double t1, double th[2]) = 0;
  virtual int info(hlbm_info *o) = 0;
  virtual int stencil(int kmax, int32_t *nbr, double *S, double *C) = 0;
  virtual int timing(int on) = 0;
  virtual int timing_get(int kernel, double *ms, int64_t *count) = 0;
  virtual int adjoint(const double *dJ, int64_t n, double grad[3]) = 0;
  // case `id` of a handle (the handle itself for a single case)
  virtual CaseBase *sub(int id) { return id == 0 ? this : nullptr; }
  virtual int set_motion(int case_id, const hlbm_motion *m) {
    (void)case_id;
    (void)m;
    err = "coupled motion applies to single cases";
    return HLBM_E_UNSUPPORTED;
  }
  virtual int set_deformation(double B, double phi) {
    (void)B;
    (void)phi;
    err = "deformation applies to single cases on a given triangulation";
    return HLBM_E_UNSUPPORTED;
  }
  virtual int tune(int trial_steps, hlbm_tuning *t) {
    (void)trial_steps;
    (void)t;
    err = "tuning applies to batched handles (ncases > 1)";
    return HLBM_E_UNSUPPORTED;
  }
  std::string err;
};

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      err = std::string(#expr) + ": " + hipGetErrorString(e_);                         \
      return HLBM_E_HIP;                                                              \
    }                                                                                 \
  } while (0)

// a checked copy: a refused one names the cause
#define COPYCHK(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) {                                                           \
      err = copy_fault_ ? std::string("refused a device copy that leaves its allocation: ") + #expr \
                        : std::string(#expr) + ": " + hipGetErrorString(e_);          \
      return HLBM_E_HIP;                                                              \
    }                                                                                 \
  } while (0)

// an unstructured grid as given to hlbm_create_mesh
struct MeshInput {
  int nnode;
  const double *xy;
  const int *type;
  int ntri;
  const int *tri;
};

inline bool valid_lattice_shape(const hlbm_tuning &t) {
  return t.lattice_threads >= 64 && t.lattice_threads <= 256 && t.lattice_threads % 64 == 0 &&
         (t.lattice_rows == 1 || t.lattice_rows == 2 || t.lattice_rows == 4);
}

template <class T, class R>
class Case final : public CaseBase {
 public:
  ~Case() override { release(); }

  // two_step: allow the two-step stream-collide (single cases; a batch
  // advances its members with the case-batched kernels)
  // gx, gy (optional): local x of each grid column and y of each row of a
  // graded grid (hlbm_create_graded)
  // mesh (optional): an unstructured grid (hlbm_create_mesh)
  int init(const hlbm_config &c, bool two_step = true, const double *gx = nullptr, const double *gy = nullptr,
           const MeshInput *mesh = nullptr) {
    cfg_ = c;
    d_ = derive(c, mesh != nullptr);
    h_ = c.h_u > 0.0 ? c.h_u : 1.0;
    has_grid_ = c.nux > 0 || c.nuy > 0 || mesh;
    body_ = has_grid_ && c.b > 0.0 && !(c.flags & HLBM_FLAG_NO_BODY);
    nodes_ = (size_t)c.nx * c.ny;
    plane_ = lattice_plane(c.nx, c.ny);
    // the grid's local extents (the same expressions as the node positions)
    gex0_ = (double)(0 - c.nux / 2) * h_;
    gex1_ = (double)(c.nux - 1 - c.nux / 2) * h_;
    gey0_ = (0.0 - 0.5 * (double)(c.nuy - 1)) * h_;
    gey1_ = ((double)(c.nuy - 1) - 0.5 * (double)(c.nuy - 1)) * h_;
    if (gx) {
      gx_.assign(gx, gx + c.nux);
      gy_.assign(gy, gy + c.nuy);
      gex0_ = gx[0];
      gex1_ = gx[c.nux - 1];
      gey0_ = gy[0];
      gey1_ = gy[c.nuy - 1];
    }
    if (has_grid_) {
      std::string e;
      const bool ok = mesh ? build_mesh(mesh->nnode, mesh->xy, mesh->type, mesh->ntri, mesh->tri, c.b, c.thickness,
                                        body_, &grid_, &e)
                           : build_grid(c.nux, c.nuy, h_, c.b, body_, &grid_, &e, gx, gy);
      if (!ok) {
        err = e;
        return HLBM_E_ARG;
      }
      if (mesh) {
        gex0_ = grid_.ex0;
        gex1_ = grid_.ex1;
        gey0_ = grid_.ey0;
        gey1_ = grid_.ey1;
      }
    }
    HIPCHK((Kernels<T, R>::prepare()));
    HIPCHK(hipGetDevice(&dev_));
    HIPCHK(hipStreamCreateWithFlags(&s_main_, hipStreamNonBlocking));
    // The grid path may run on a second stream, concurrently with the
    // lattice update; measured on MI355X it is faster on the same stream
    // (the latency-bound sub-steps slow down under the lattice kernel's HBM
    // traffic), so a second stream is opt-in.
    if (std::getenv("HLBM_TWO_STREAMS")) HIPCHK(hipStreamCreateWithFlags(&s_grid_, hipStreamNonBlocking));
    else s_grid_ = s_main_;
    HIPCHK(hipEventCreateWithFlags(&ev_fork_, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ev_join_, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ev_flag_, hipEventDisableTiming));
    HIPCHK(hipHostMalloc((void **)&hflag_, sizeof(int), hipHostMallocDefault));
    *hflag_ = 0;
    HIPCHK(alloc(&lat_[0], 9 * plane_ * sizeof(T)));
    HIPCHK(alloc(&lat_[1], 9 * plane_ * sizeof(T)));
    lat_base_ = lat_[0];
    use_graphs_ = std::getenv("HLBM_NO_GRAPHS") == nullptr;
    const int64_t cap = std::max<int64_t>(c.max_steps, 1);
    HIPCHK(alloc(&hist_, 2 * cap * sizeof(double)));
    HIPCHK(alloc(&dk_, sizeof(int64_t)));
    HIPCHK(alloc(&flag_, sizeof(int)));
    HIPCHK(alloc(&counts_, 2 * sizeof(unsigned long long)));
    HIPCHK(alloc(&done_, sizeof(unsigned)));
    HIPCHK(alloc(&dk_copy_, sizeof(int64_t)));
    HIPCHK(hipMemset(dk_copy_, 0, sizeof(int64_t)));
    HIPCHK(hipMemset(done_, 0, sizeof(unsigned)));
    HIPCHK(hipMemset(dk_, 0, sizeof(int64_t)));
    HIPCHK(hipMemset(flag_, 0, sizeof(int)));
    HIPCHK(hipMemset(counts_, 0, 2 * sizeof(unsigned long long)));
    HIPCHK(hipMemset(hist_, 0, 2 * cap * sizeof(double)));
    const int N = has_grid_ ? grid_.nnode : 0;
    if (has_grid_) {
      for (int i = 0; i < 2; ++i) HIPCHK(alloc(&gbuf_[i], 9 * (size_t)N * sizeof(R)));
      HIPCHK(alloc(&star_f_, 9 * (size_t)N * sizeof(R)));
      HIPCHK(alloc(&star_n_, 9 * (size_t)N * sizeof(R)));
      HIPCHK(hipMemset(star_f_, 0, 9 * (size_t)N * sizeof(R)));
      HIPCHK(hipMemset(star_n_, 0, 9 * (size_t)N * sizeof(R)));
      if (grid_.mesh) {
        auto conv = [](const std::vector<double> &a) { return std::vector<R>(a.begin(), a.end()); };
        const std::vector<R> mC = conv(grid_.C), mGx = conv(grid_.Gx), mGy = conv(grid_.Gy);
        HIPCHK(upload(&m_row_, grid_.row.data(), grid_.row.size() * sizeof(int)));
        HIPCHK(upload(&m_col_, grid_.col.data(), grid_.col.size() * sizeof(int)));
        HIPCHK(upload(&m_C_, mC.data(), mC.size() * sizeof(R)));
        HIPCHK(upload(&m_Gx_, mGx.data(), mGx.size() * sizeof(R)));
        HIPCHK(upload(&m_Gy_, mGy.data(), mGy.size() * sizeof(R)));
        HIPCHK(upload(&m_x_, grid_.x.data(), grid_.x.size() * sizeof(double)));
        HIPCHK(upload(&m_y_, grid_.y.data(), grid_.y.size() * sizeof(double)));
        HIPCHK(upload(&m_type_, grid_.type.data(), grid_.type.size() * sizeof(int)));
        HIPCHK(upload(&m_tri_, grid_.tri.data(), grid_.tri.size() * sizeof(int)));
        HIPCHK(upload(&m_txy_, grid_.txy.data(), grid_.txy.size() * sizeof(double)));
        HIPCHK(upload(&m_bstart_, grid_.bstart.data(), grid_.bstart.size() * sizeof(int)));
        HIPCHK(upload(&m_blist_, grid_.blist.data(), std::max<size_t>(1, grid_.blist.size()) * sizeof(int)));
      }
      std::vector<GridClass<R>> tab(grid_.classes.size());
      for (size_t i = 0; i < tab.size(); ++i) {
        const GridClass<double> &g = grid_.classes[i];
        GridClass<R> &t = tab[i];
        std::memset(&t, 0, sizeof(t));
        t.type = g.type;
        for (int s = 0; s < NSLOT; ++s) {
          t.C[s] = (R)g.C[s];
          t.Gx[s] = (R)g.Gx[s];
          t.Gy[s] = (R)g.Gy[s];
        }
        auto zero = [&](int s) { return t.C[s] == R(0) && t.Gx[s] == R(0) && t.Gy[s] == R(0); };
        t.zero_diag = (zero(2) && zero(6) ? kZeroDiag26 : 0) | (zero(0) && zero(8) ? kZeroDiag08 : 0);
      }
      if (!grid_.mesh) {
        HIPCHK(upload(&tab_, tab.data(), tab.size() * sizeof(GridClass<R>)));
        // node codes: 16 class + 4 zero_diag + type (static: the grid moves rigidly)
        std::vector<int> code(grid_.cls.size());
        for (size_t p = 0; p < code.size(); ++p) {
          const int k = grid_.cls[p];
          code[p] = k >= 0 ? 16 * k + 4 * tab[k].zero_diag + tab[k].type : -1;
        }
        HIPCHK(upload(&ncode_, code.data(), code.size() * sizeof(int)));
      }
      HIPCHK(upload(&iface_, grid_.iface.data(), grid_.iface.size() * sizeof(int)));
      HIPCHK(upload(&wall_, grid_.wall.data(), grid_.wall.size() * sizeof(WallEdge)));
      if (!gx_.empty()) {
        HIPCHK(upload(&dgx_, gx_.data(), gx_.size() * sizeof(double)));
        HIPCHK(upload(&dgy_, gy_.data(), gy_.size() * sizeof(double)));
      }
      // per-step scalars for k = 0 .. max_steps, wall velocity per sub-step
      std::vector<StepParams> &P = P_host_;
      P.resize(cap + 1);
      for (int64_t k = 0; k <= cap; ++k) P[k] = params_at(k);
      HIPCHK(upload(&params_, P.data(), P.size() * sizeof(StepParams)));
      std::vector<R> uw((size_t)cap * d_.n);
      for (int64_t k = 0; k < cap; ++k)
        for (int m = 0; m < d_.n; ++m) {
          const double t = (double)k + (double)(m + 1) / (double)d_.n;
          uw[(size_t)k * d_.n + m] = (R)(d_.A * d_.omega * std::cos(d_.omega * t));
        }
      HIPCHK(upload(&uw_, uw.data(), uw.size() * sizeof(R)));
      int x0 = P[0].ix0, x1 = P[0].ix1;
      k2_x0_ = x0;
      k2_w_ = std::max(1, x1 - x0 + 1);
      int hmax = 1;
      for (int64_t k = 0; k <= cap; ++k)
        hmax = std::max(hmax, std::max(P[k].iy1, P[k].piy1) - std::min(P[k].iy0, P[k].piy0) + 1);
      k2_h_ = hmax;
      if (c.ckpt_every > 0) {
        // checkpoints of (lattice, grid) at every multiple of ckpt_every
        ckW_ = c.ckpt_every;
        nck_ = cap / ckW_ + 1;
        ck_lat_bytes_ = 9 * plane_ * sizeof(T);
        ck_grid_bytes_ = 9 * (size_t)N * sizeof(R);
        HIPCHK(alloc(&ck_lat_, (size_t)nck_ * ck_lat_bytes_));
        HIPCHK(alloc(&ck_grid_, (size_t)nck_ * ck_grid_bytes_));
      }
    }
    two_step_ = two_step && std::getenv("HLBM_ONE_STEP") == nullptr && choose_band();
    if (two_step_) {
      HIPCHK(alloc(&lat_[2], 9 * plane_ * sizeof(T)));
      Kernels<T, R>::fill_rest((T *)lat_[2], plane_, nullptr, 0, s_main_);
    }
    for (int i = 0; i < 3; ++i) phys_[i] = lat_[i];
    Kernels<T, R>::fill_rest((T *)lat_[0], plane_, has_grid_ ? (R *)gbuf_[0] : nullptr, N, s_main_);
    Kernels<T, R>::fill_rest((T *)lat_[1], plane_, has_grid_ ? (R *)gbuf_[1] : nullptr, N, s_main_);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s_main_));
    return HLBM_OK;
  }

#define ENQ(expr)                  \
  do {                             \
    e = (expr);                    \
    if (e != hipSuccess) return e; \
  } while (0)

  // Enqueue one structured step t_k -> t_{k+1} (host bookkeeping included).
  // Stream-collide with its own start and end events when timing is on
  // (the events are taken at the kernel's own start and end on its stream).
  // donors: the launch also computes the grid path's interface donors
  void stream_collide_timed(const CaseView<T, R> &v, bool donors = false) {
    if (timing_ == 1 || timing_ == 2) {
      Kernels<T, R>::stream_collide(v, s_main_, tev_[tslot_][8], tev_[tslot_][2], lattice_threads_, lattice_rows_,
                                    lattice_order_, donors);
    } else {
      Kernels<T, R>::stream_collide(v, s_main_, nullptr, nullptr, lattice_threads_, lattice_rows_, lattice_order_,
                                    donors);
    }
  }

  hipError_t enqueue_step() {
    hipError_t e = hipSuccess;
    CaseView<T, R> v = view();
    if (timing_ == 1) ENQ(hipEventRecord(tev_[tslot_][0], s_main_));
    if (has_grid_) {
      // 0. a bending grid takes the configuration of t_k
      if (deform_) Kernels<T, R>::mesh_deform(deform_view(), s_main_);
      // 1. lattice interpolation nodes from the grid at t_k, Eq.(postcollision2_s)
      Kernels<T, R>::lattice_from_grid(v, (const R *)gbuf_[gcur_], s_main_);
      if (timing_ == 1) ENQ(hipEventRecord(tev_[tslot_][1], s_main_));
      if (s_grid_ != s_main_) {
        ENQ(hipEventRecord(ev_fork_, s_main_));
        ENQ(hipStreamWaitEvent(s_grid_, ev_fork_, 0));
      }
      // 2. lattice stream-collide, Eq.(LBE); on one stream (and unless the
      // donors are timed apart) it also computes step 3's donors, which
      // read the same source lattice
      const bool fuse = s_grid_ == s_main_ && timing_ != 1;
      stream_collide_timed(v, fuse);
      // 3.-6. grid path: donors, n sub-steps, refill, force
      ENQ(enqueue_grid_path(v, fuse));
      if (s_grid_ != s_main_) {
        ENQ(hipEventRecord(ev_join_, s_grid_));
        ENQ(hipStreamWaitEvent(s_main_, ev_join_, 0));
      }
    } else {
      if (timing_ == 1) ENQ(hipEventRecord(tev_[tslot_][1], s_main_));
      stream_collide_timed(v);
    }
    if (timing_ == 1) ENQ(hipEventRecord(tev_[tslot_][7], s_main_));
    if (timing_) ++tslot_;
    ENQ(hipGetLastError());
    std::swap(lat_[0], lat_[1]);
    ++k_;
    return hipSuccess;
  }

  // Grid path of the step whose lattice (post-collision at t_k) v.A holds:
  // donors (unless the lattice launch computed them), n sub-steps, refill,
  // force (steps 3-6 of the step).
  hipError_t enqueue_grid_path(const CaseView<T, R> &v, bool donors_done = false) {
    hipError_t e = hipSuccess;
    if (timing_ == 1) ENQ(hipEventRecord(tev_[tslot_][3], s_grid_));
    if (!donors_done) Kernels<T, R>::interface_donors(v, s_grid_);
    int cur = gcur_;
    const int blk = substep_block(substep_variant_);
    // level 3: every sub-step launch of the step (up to kTimedLaunches),
    // once per timing slot
    const bool time_sub = timing_ == 3 && sub_mark_ != tslot_;
    if (time_sub) {
      sub_mark_ = tslot_;
      sub_n_[tslot_] = 0;
    }
    auto sub_ev = [&](int which) -> hipEvent_t {  // 0: start, 1: end of the next timed launch
      if (!time_sub || sub_n_[tslot_] >= kTimedLaunches) return nullptr;
      hipEvent_t ev = tev3_[tslot_][2 * sub_n_[tslot_] + which];
      if (which == 1) ++sub_n_[tslot_];
      return ev;
    };
    if (grid_.mesh) {  // one sub-step per launch
      for (int m = 0; m < d_.n; ++m) {
        hipEvent_t e0 = sub_ev(0), e1 = sub_ev(1);
        Kernels<T, R>::mesh_substep(v, (const R *)gbuf_[cur], (R *)gbuf_[1 - cur], m, s_grid_, e0, e1);
        cur = 1 - cur;
      }
    } else {
      for (int m = 0; m < d_.n; m += blk) {
        const int cnt = std::min(blk, d_.n - m);
        hipEvent_t e0 = sub_ev(0), e1 = sub_ev(1);
        Kernels<T, R>::grid_substeps(v, (const R *)gbuf_[cur], (R *)gbuf_[1 - cur], m, cnt, s_grid_, nullptr,
                                     nullptr, nullptr, 0, substep_variant_, e0, e1);
        cur = 1 - cur;
      }
    }
    if (timing_ == 1) ENQ(hipEventRecord(tev_[tslot_][4], s_grid_));
    if (fsi_) {
      // coupled motion: the force gives y_{k+1}, which the refill needs
      Kernels<T, R>::force(v, (const R *)gbuf_[cur], s_grid_, 0);
      Kernels<T, R>::refill(v, (const R *)gbuf_[cur], (R *)gbuf_[1 - cur], s_grid_);
      Kernels<T, R>::advance_step(v, s_grid_);
    } else if (timing_ != 1) {  // one launch (level 1 times the two apart)
      Kernels<T, R>::refill_force(v, (const R *)gbuf_[cur], (R *)gbuf_[1 - cur], done_, s_grid_);
    } else {
      Kernels<T, R>::refill(v, (const R *)gbuf_[cur], (R *)gbuf_[1 - cur], s_grid_);
      if (timing_ == 1) ENQ(hipEventRecord(tev_[tslot_][5], s_grid_));
      Kernels<T, R>::force(v, (const R *)gbuf_[cur], s_grid_);
    }
    if (timing_ == 1) ENQ(hipEventRecord(tev_[tslot_][6], s_grid_));
    gcur_ = 1 - cur;
    return e;
  }

  // Two structured steps t_k -> t_{k+2}. Outside the band the lattice takes
  // both steps in one launch (A -> C); the band takes the first step there
  // too (into B), and after step k's grid path and step k+1's interpolation
  // nodes, its second step with the single-step kernel (B -> C, on the band
  // only). Every node computes what two single steps compute, in the same
  // arithmetic. Afterwards C holds t_{k+2}.
  hipError_t enqueue_pair() {
    hipError_t e = hipSuccess;
    CaseView<T, R> v = view();
    const bool two = s_grid_ != s_main_;  // the grid path on its own stream
    auto fork = [&]() -> hipError_t {
      hipError_t r = hipEventRecord(ev_fork_, s_main_);
      return r == hipSuccess ? hipStreamWaitEvent(s_grid_, ev_fork_, 0) : r;
    };
    auto join = [&]() -> hipError_t {
      hipError_t r = hipEventRecord(ev_join_, s_grid_);
      return r == hipSuccess ? hipStreamWaitEvent(s_main_, ev_join_, 0) : r;
    };
    if (has_grid_) {
      if (deform_) Kernels<T, R>::mesh_deform(deform_view(), s_main_);
      Kernels<T, R>::lattice_from_grid(v, (const R *)gbuf_[gcur_], s_main_);
    }
    // step k's grid path reads only the lattice of t_k: it may run beside
    // the two-step launch, which then reads a copy of the step counter (the
    // grid path advances it)
    if (has_grid_ && two) {
      Kernels<T, R>::copy_step(dk_, dk_copy_, s_main_);
      v.dkl = dk_copy_;
      ENQ(fork());
    }
    // on one stream the lattice launches also compute the donors of the grid
    // path that follows them (both read only the lattice of t_k or t_{k+1})
    const bool fuse = has_grid_ && !two;
    if (timing_ == 2)
      Kernels<T, R>::stream_collide2(v, s_main_, tev_[tslot_][8], tev_[tslot_][2], two_step_order_, fuse);
    else Kernels<T, R>::stream_collide2(v, s_main_, nullptr, nullptr, two_step_order_, fuse);
    if (has_grid_) {
      ENQ(enqueue_grid_path(v, fuse));
      if (two) ENQ(join());
      CaseView<T, R> w = view();
      w.A = (const T *)lat_[1];
      w.B = (T *)lat_[2];
      w.wx0 = band_[0];
      w.ww = band_[1] - band_[0] + 1;
      w.wy0 = band_[2];
      w.wh = band_[3] - band_[2] + 1;
      // (step k's refill and force have read the configuration of t_k)
      if (deform_) Kernels<T, R>::mesh_deform(deform_view(), s_main_);
      Kernels<T, R>::lattice_from_grid(w, (const R *)gbuf_[gcur_], s_main_);
      // step k+1's grid path and the band's second step both read t_{k+1}
      if (two) ENQ(fork());
      Kernels<T, R>::stream_collide(w, s_main_, nullptr, nullptr, lattice_threads_, lattice_rows_, 0, fuse);
      ENQ(enqueue_grid_path(w, fuse));
      if (two) ENQ(join());
    }
    if (timing_) ++tslot_;
    ENQ(hipGetLastError());
    void *a = lat_[0], *b = lat_[1];
    lat_[0] = lat_[2];
    lat_[1] = a;
    lat_[2] = b;
    k_ += 2;
    return hipSuccess;
  }

  // n steps: pairs on the two-step path where it is on, single steps
  // otherwise (and for an odd last step)
  hipError_t enqueue_steps(int n, int *done) {
    *done = 0;
    while (*done < n) {
      hipError_t e;
      if (two_step_ && timing_ != 1 && n - *done >= 2) {
        e = enqueue_pair();
        if (e == hipSuccess) *done += 2;
      } else {
        e = enqueue_step();
        if (e == hipSuccess) *done += 1;
      }
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }

  // which physical lattice buffer each role holds, and the grid buffer
  int layout_key() const {
    int i0 = 0, i1 = 0;
    for (int i = 0; i < 3; ++i) {
      if (lat_[0] == phys_[i]) i0 = i;
      if (lat_[1] == phys_[i]) i1 = i;
    }
    return (3 * i0 + i1) * 2 + gcur_;
  }

  // kGraphSteps steps captured as one HIP graph per buffer arrangement:
  // kernels read the step index from device memory, so a graph replays for
  // every later kGraphSteps steps that start from the same arrangement.
  hipError_t graph_for_current_layout(hipGraphExec_t *out) {
    const int key = layout_key();
    if (gexec_[key]) {
      *out = gexec_[key];
      return hipSuccess;
    }
    void *l0 = lat_[0], *l1 = lat_[1], *l2 = lat_[2];
    const int g0 = gcur_;
    const int64_t k0 = k_;
    hipError_t e = hipStreamBeginCapture(s_main_, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    int n = 0;
    hipError_t e2 = enqueue_steps(kGraphSteps, &n);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s_main_, &g);
    after_graph_[key][0] = lat_[0];
    after_graph_[key][1] = lat_[1];
    after_graph_[key][2] = lat_[2];
    after_gcur_[key] = gcur_;
    lat_[0] = l0;
    lat_[1] = l1;
    lat_[2] = l2;
    gcur_ = g0;
    k_ = k0;
    if (e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return e2;
    }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&gexec_[key], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
    *out = gexec_[key];
    return hipSuccess;
  }

  int step(int64_t nsteps) override {
    const int rc = enqueue_run(nsteps);
    if (rc != HLBM_OK) return rc;
    return sync();
  }

  // the steps enqueued; the flag of those that have finished (read from the
  // copy a previous call enqueued, if it is done) is checked without waiting
  int step_async(int64_t nsteps) override {
    if (timing_) return step(nsteps);  // timed steps are harvested on the host
    const int rc = enqueue_run(nsteps);
    if (rc != HLBM_OK) return rc;
    pending_ = true;
    int seen = 0;
    if (flag_copied_) {
      const hipError_t q = hipEventQuery(ev_flag_);
      if (q == hipSuccess) seen = *hflag_;
      else if (q != hipErrorNotReady) HIPCHK(q);
    }
    HIPCHK(hipMemcpyAsync(hflag_, flag_, sizeof(int), hipMemcpyDeviceToHost, s_main_));
    HIPCHK(hipEventRecord(ev_flag_, s_main_));
    flag_copied_ = true;
    return flag_status(seen);
  }

  int sync() override {
    HIPCHK(hipStreamSynchronize(s_main_));
    pending_ = false;
    int flag = 0;
    HIPCHK(hipMemcpy(&flag, flag_, sizeof(int), hipMemcpyDeviceToHost));
    return flag_status(flag);
  }

  void drain() override {
    if (pending_) (void)hipStreamSynchronize(s_main_);
    pending_ = false;
  }

  int flag_status(int flag) {
    if (flag & 4) return fail(HLBM_E_UNSTABLE, "a lattice node to interpolate lies outside the grid");
    if (flag & 2) return fail(HLBM_E_UNSTABLE, "a density became non-positive or not a number");
    if (flag) return fail(HLBM_E_UNSTABLE, has_grid_ ? "non-finite force on the lamina" : "unstable");
    return HLBM_OK;
  }

  // enqueue nsteps steps (graphs, pairs or single steps) on the main stream
  int enqueue_run(int64_t nsteps) {
    if (nsteps < 0) return fail(HLBM_E_ARG, "nsteps < 0");
    if (has_grid_ && k_ + nsteps > cfg_.max_steps) return fail(HLBM_E_ARG, "force history would exceed max_steps");
    int64_t done = 0;
    while (done < nsteps) {
      int64_t room = nsteps - done;
      if (ckW_ > 0) {
        if (k_ % ckW_ == 0 && k_ / ckW_ < nck_) {
          const size_t w = (size_t)(k_ / ckW_);
          COPYCHK(copy_checked((char *)ck_lat_ + w * ck_lat_bytes_, lat_[0], ck_lat_bytes_,
                               hipMemcpyDeviceToDevice, s_main_));
          COPYCHK(copy_checked((char *)ck_grid_ + w * ck_grid_bytes_, gbuf_[gcur_], ck_grid_bytes_,
                               hipMemcpyDeviceToDevice, s_main_));
        }
        room = std::min<int64_t>(room, ckW_ - k_ % ckW_);
      }
      if (!timing_ && use_graphs_ && room >= kGraphSteps) {
        hipGraphExec_t ge = nullptr;
        HIPCHK(graph_for_current_layout(&ge));
        HIPCHK(hipGraphLaunch(ge, s_main_));
        // the buffer arrangement the captured steps end in
        const int key = layout_key();
        lat_[0] = after_graph_[key][0];
        lat_[1] = after_graph_[key][1];
        lat_[2] = after_graph_[key][2];
        gcur_ = after_gcur_[key];
        k_ += kGraphSteps;
        done += kGraphSteps;
      } else {
        int n = 0;
        HIPCHK(enqueue_steps(room >= 2 && timing_ != 1 ? 2 : 1, &n));
        if (timing_ && tslot_ == kTimingRing) HIPCHK(harvest());
        done += n;
      }
    }
    if (timing_ && tslot_ > 0) HIPCHK(harvest());
    return HLBM_OK;
  }

  int get_state(int which, void *buf, size_t bytes) override {
    HIPCHK(hipStreamSynchronize(s_main_));
    if (which == HLBM_STATE_LATTICE) {
      if (bytes != 9 * nodes_ * sizeof(double)) return fail(HLBM_E_ARG, "lattice state size mismatch");
      double *tmp = nullptr;
      HIPCHK(hipMalloc(&tmp, bytes));
      Kernels<T, R>::lattice_to_f64((const T *)lat_[0], tmp, plane_, nodes_, s_main_);
      hipError_t e = hipMemcpyAsync(buf, tmp, bytes, hipMemcpyDeviceToHost, s_main_);
      if (e == hipSuccess) e = hipStreamSynchronize(s_main_);
      (void)hipFree(tmp);
      HIPCHK(e);
      return HLBM_OK;
    }
    if (which == HLBM_STATE_GRID) {
      if (!has_grid_) return fail(HLBM_E_STATE, "case has no grid");
      const size_t n = 9 * (size_t)grid_.nnode;
      if (bytes != n * sizeof(double)) return fail(HLBM_E_ARG, "grid state size mismatch");
      std::vector<R> tmp(n);
      HIPCHK(hipMemcpy(tmp.data(), gbuf_[gcur_], n * sizeof(R), hipMemcpyDeviceToHost));
      double *out = (double *)buf;
      for (size_t i = 0; i < n; ++i) out[i] = (double)tmp[i];
      return HLBM_OK;
    }
    if (which == HLBM_STATE_MOTION) {
      if (!fsi_) return fail(HLBM_E_STATE, "case has prescribed motion");
      if (bytes != 2 * (size_t)k_ * sizeof(double)) return fail(HLBM_E_ARG, "motion state size mismatch");
      if (k_ > 0) HIPCHK(hipMemcpy(buf, mstate_ + 2, bytes, hipMemcpyDeviceToHost));
      return HLBM_OK;
    }
    if (which == HLBM_STATE_ADJ_LATTICE || which == HLBM_STATE_ADJ_GRID) {
      if (!adj_done_) return fail(HLBM_E_STATE, "no adjoint has been run");
      const bool lat = which == HLBM_STATE_ADJ_LATTICE;
      // lattice: [9][plane] on the device, [9][ny][nx] for the caller
      const size_t per = lat ? nodes_ : (size_t)grid_.nnode, stride = lat ? plane_ : per;
      if (bytes != 9 * per * sizeof(double)) return fail(HLBM_E_ARG, "adjoint state size mismatch");
      std::vector<R> tmp(9 * stride);
      HIPCHK(hipMemcpy(tmp.data(), lat ? (void *)alat_[adj_lc_] : (void *)agrid_[adj_gc_], 9 * stride * sizeof(R),
                       hipMemcpyDeviceToHost));
      double *out = (double *)buf;
      for (int q = 0; q < 9; ++q)
        for (size_t i = 0; i < per; ++i) out[q * per + i] = (double)tmp[q * stride + i];
      return HLBM_OK;
    }
    return fail(HLBM_E_ARG, "unknown state selector");
  }

  // The lattice or grid state as get_state returns it, converted to FP64 a
  // piece at a time in the static staging buffer instead of an allocated one.
  int get_state_noalloc(int which, void *buf, size_t bytes) override {
    if (which != HLBM_STATE_LATTICE && which != HLBM_STATE_GRID)
      return fail(HLBM_E_ARG, "only the lattice and grid states are read without allocating");
    if (which == HLBM_STATE_GRID && !has_grid_) return fail(HLBM_E_STATE, "case has no grid");
    const bool lat = which == HLBM_STATE_LATTICE;
    const size_t per = lat ? nodes_ : (size_t)grid_.nnode, stride = lat ? plane_ : per;
    if (bytes != 9 * per * sizeof(double)) return fail(HLBM_E_ARG, lat ? "lattice state size mismatch" : "grid state size mismatch");
    double *sc = nullptr;
    HIPCHK(scratch_on(dev_, &sc));
    HIPCHK(hipStreamSynchronize(s_main_));
    const T *L = (const T *)lat_[0];
    const R *G = has_grid_ ? (const R *)gbuf_[gcur_] : nullptr;
    HIPCHK(stage_planes((double *)buf, per, sc, kScratchElems, s_main_, [&](int q, size_t a, size_t n, double *dst) {
      if (lat) Kernels<T, R>::lattice_stage_f64(L + (size_t)q * stride + a, dst, n, q, s_main_);
      else Kernels<T, R>::grid_stage_f64(G + (size_t)q * stride + a, dst, n, s_main_);
    }));
    return HLBM_OK;
  }

  int set_state(int which, const void *buf, size_t bytes) override {
    HIPCHK(hipStreamSynchronize(s_main_));
    if (which != HLBM_STATE_LATTICE && which != HLBM_STATE_GRID) return fail(HLBM_E_ARG, "state cannot be set");
    if (k_ > 0) ck_valid_ = false;
    if (which == HLBM_STATE_LATTICE) {
      if (bytes != 9 * nodes_ * sizeof(double)) return fail(HLBM_E_ARG, "lattice state size mismatch");
      double *tmp = nullptr;
      HIPCHK(hipMalloc(&tmp, bytes));
      hipError_t e = hipMemcpyAsync(tmp, buf, bytes, hipMemcpyHostToDevice, s_main_);
      if (e == hipSuccess) {
        Kernels<T, R>::lattice_from_f64(tmp, (T *)lat_[0], plane_, nodes_, s_main_);
        e = hipStreamSynchronize(s_main_);
      }
      (void)hipFree(tmp);
      HIPCHK(e);
      return HLBM_OK;
    }
    if (which == HLBM_STATE_GRID) {
      if (!has_grid_) return fail(HLBM_E_STATE, "case has no grid");
      const size_t n = 9 * (size_t)grid_.nnode;
      if (bytes != n * sizeof(double)) return fail(HLBM_E_ARG, "grid state size mismatch");
      std::vector<R> tmp(n);
      const double *in = (const double *)buf;
      for (size_t i = 0; i < n; ++i) tmp[i] = (R)in[i];
      HIPCHK(hipMemcpy(gbuf_[gcur_], tmp.data(), n * sizeof(R), hipMemcpyHostToDevice));
      return HLBM_OK;
    }
    return fail(HLBM_E_ARG, "unknown state selector");
  }

  // Single-harmonic least-squares fit of F_y (Sec. 2.1) and Theta from
  // Eq.(force_phasor): a_s + i a_c = (pi/4) rho omega^2 L^2 A Theta, rho = 1.
  int force(double *hist, int64_t cap, int64_t *n_out, double t0, double t1, double th[2]) override {
    HIPCHK(hipStreamSynchronize(s_main_));
    const int64_t n = has_grid_ ? k_ : 0;
    std::vector<double> hbuf(2 * std::max<int64_t>(n, 1));
    if (n > 0) HIPCHK(hipMemcpy(hbuf.data(), hist_, 2 * n * sizeof(double), hipMemcpyDeviceToHost));
    if (th) {
      if (!(d_.omega > 0.0)) return fail(HLBM_E_ARG, "no oscillation to fit");
      const double period = 2.0 * M_PI / d_.omega;
      double ss = 0, sc = 0, cc = 0, sf = 0, cf = 0;
      int64_t cnt = 0;
      for (int64_t k = 0; k < n; ++k) {
        const double t = (double)(k + 1);
        if (t < t0 * period || t >= t1 * period) continue;
        const double sn = std::sin(d_.omega * t), cs = std::cos(d_.omega * t), F = hbuf[2 * k + 1];
        ss += sn * sn;
        sc += sn * cs;
        cc += cs * cs;
        sf += sn * F;
        cf += cs * F;
        ++cnt;
      }
      const double det = ss * cc - sc * sc;
      if (cnt < 2 || !(std::fabs(det) > 0.0)) return fail(HLBM_E_ARG, "fit window holds fewer than two samples");
      const double norm = 0.25 * M_PI * d_.omega * d_.omega * cfg_.b * cfg_.b * d_.A;
      th[0] = (sf * cc - cf * sc) / det / norm;
      th[1] = (cf * ss - sf * sc) / det / norm;
    }
    if (hist) std::memcpy(hist, hbuf.data(), 2 * std::min(cap, n) * sizeof(double));
    if (n_out) *n_out = n;
    return HLBM_OK;
  }

  int info(hlbm_info *o) override {
    std::memset(o, 0, sizeof(*o));
    o->nu = d_.nu;
    o->tau_u = d_.tau_u;
    o->dt_u = 1.0 / (double)d_.n;
    o->A = d_.A;
    o->omega = d_.omega;
    o->period = d_.omega > 0.0 ? 2.0 * M_PI / d_.omega : 0.0;
    o->u_max = d_.A * d_.omega;
    o->mach = o->u_max * std::sqrt(3.0);
    o->reynolds = d_.nu > 0.0 ? o->u_max * cfg_.b / d_.nu : 0.0;
    o->eps = cfg_.b > 0.0 ? d_.A / cfg_.b : 0.0;
    o->beta_limit_ok = o->eps > 0.0 ? (cfg_.beta < 2.6 * std::pow(o->eps, -1.6)) : 1;
    o->n_sub = d_.n;
    o->step = k_;
    o->y = d_.A * std::sin(d_.omega * (double)k_);
    if (fsi_) {
      HIPCHK(hipStreamSynchronize(s_main_));
      HIPCHK(hipMemcpy(&o->y, mstate_ + 2 * k_, sizeof(double), hipMemcpyDeviceToHost));
    }
    o->lattice_bytes = (int64_t)(9 * plane_ * sizeof(T));
    o->two_step = two_step_ ? 1 : 0;
    {
      int flag = 0;
      HIPCHK(hipMemcpy(&flag, flag_, sizeof(int), hipMemcpyDeviceToHost));
      o->status = flag ? HLBM_STATUS_UNSTABLE : (has_grid_ && k_ >= cfg_.max_steps ? HLBM_STATUS_DONE : HLBM_STATUS_RUNNING);
    }
    if (has_grid_) {
      o->nnode = grid_.nnode;
      o->ntri = grid_.ntri;
      o->n_interface = (int)grid_.iface.size();
      o->n_wall_edges = (int)grid_.wall.size();
      o->n_classes = (int)grid_.classes.size();
      for (int t : grid_.type) o->n_wall += (t == NODE_WALL);
      unsigned long long cnt[2];
      HIPCHK(hipStreamSynchronize(s_main_));
      HIPCHK(hipMemcpy(cnt, counts_, sizeof(cnt), hipMemcpyDeviceToHost));
      o->n_type1 = (int64_t)cnt[0];
      o->n_type2 = (int64_t)cnt[1];
      o->n_type3 = k_ * (int64_t)(grid_.nnode - o->n_wall) - o->n_type1 - o->n_type2;
    }
    return HLBM_OK;
  }

  int stencil(int kmax, int32_t *nbr, double *S, double *C) override {
    if (!has_grid_) return fail(HLBM_E_STATE, "case has no grid");
    static const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    if (grid_.mesh) {  // the stored stencils, the node first
      int need = 0;
      for (int p = 0; p < grid_.nnode; ++p) need = std::max(need, grid_.row[p + 1] - grid_.row[p]);
      if (kmax < need) return fail(HLBM_E_ARG, "kmax smaller than the largest stencil");
      const std::vector<double> *Cw = &grid_.C, *Gxw = &grid_.Gx, *Gyw = &grid_.Gy;
      std::vector<double> dC, dGx, dGy;
      if (deform_) {  // a bending grid: the weights of the current configuration
        HIPCHK(hipStreamSynchronize(s_main_));
        if (s_grid_ != s_main_) HIPCHK(hipStreamSynchronize(s_grid_));
        const size_t ne = grid_.col.size();
        std::vector<R> buf(ne);
        std::vector<double> *dst[3] = {&dC, &dGx, &dGy};
        const R *src[3] = {m_C_, m_Gx_, m_Gy_};
        for (int a = 0; a < 3; ++a) {
          HIPCHK(hipMemcpy(buf.data(), src[a], ne * sizeof(R), hipMemcpyDeviceToHost));
          dst[a]->assign(buf.begin(), buf.end());
        }
        Cw = &dC;
        Gxw = &dGx;
        Gyw = &dGy;
      }
      for (int p = 0; p < grid_.nnode; ++p) {
        const int e0 = grid_.row[p], k = grid_.row[p + 1] - e0;
        for (int u = 0; u < kmax; ++u) {
          const bool in = u < k;
          if (nbr) nbr[(size_t)p * kmax + u] = in ? grid_.col[e0 + u] : -1;
          if (C) C[(size_t)p * kmax + u] = in ? (*Cw)[e0 + u] : 0.0;
          if (S)
            for (int r = 0; r < 9; ++r)
              S[((size_t)p * 9 + r) * kmax + u] = in ? cx[r] * (*Gxw)[e0 + u] + cy[r] * (*Gyw)[e0 + u] : 0.0;
        }
      }
      return HLBM_OK;
    }
    int need = 0;
    for (const auto &c : grid_.classes) {
      int k = 0;
      for (int s = 0; s < NSLOT; ++s) k += c.C[s] != 0.0;
      need = std::max(need, k);
    }
    if (kmax < need) return fail(HLBM_E_ARG, "kmax smaller than the largest stencil");
    for (int p = 0; p < grid_.nnode; ++p) {
      const GridClass<double> &c = grid_.classes[grid_.cls[p]];
      // slot order: the node itself, then the neighbours by node index
      int order[NSLOT], k = 0;
      order[k++] = SELF_SLOT;
      for (int s = 0; s < NSLOT; ++s)
        if (s != SELF_SLOT && c.C[s] != 0.0) order[k++] = s;
      for (int u = 0; u < kmax; ++u) {
        const bool in = u < k;
        const int s = in ? order[u] : 0;
        const int q = p + (s % 3 - 1) + (s / 3 - 1) * cfg_.nux;
        if (nbr) nbr[(size_t)p * kmax + u] = in ? q : -1;
        if (C) C[(size_t)p * kmax + u] = in ? c.C[s] : 0.0;
        if (S)
          for (int r = 0; r < 9; ++r)
            S[((size_t)p * 9 + r) * kmax + u] = in ? cx[r] * c.Gx[s] + cy[r] * c.Gy[s] : 0.0;
      }
    }
    return HLBM_OK;
  }

  int timing(int on) override {
    HIPCHK(hipStreamSynchronize(s_main_));
    if (on && !tev_[0][0])
      for (auto &ring : tev_)
        for (auto &e : ring) HIPCHK(hipEventCreate(&e));
    if (on == 3 && !tev3_[0][0])
      for (auto &ring : tev3_)
        for (auto &e : ring) HIPCHK(hipEventCreate(&e));
    tslot_ = 0;
    sub_mark_ = -1;
    for (int &n : sub_n_) n = 0;
    for (int i = 0; i < kTimedKernels; ++i) {
      tms_[i] = 0.0;
      tcount_[i] = 0;
    }
    if (on < 0 || on > 3) return fail(HLBM_E_ARG, "timing level must be 0, 1, 2 or 3");
    if (on == 3 && !has_grid_) return fail(HLBM_E_STATE, "timing level 3 times the grid sub-steps of a case with a grid");
    timing_ = on;
    return HLBM_OK;
  }

  int set_motion(int case_id, const hlbm_motion *m) override {
    if (case_id != 0) return fail(HLBM_E_ARG, "case_id must be 0");
    if (!m) return fail(HLBM_E_ARG, "null argument");
    if (k_ != 0) return fail(HLBM_E_STATE, "coupled motion must be set before the first step");
    if (!has_grid_ || !body_) return fail(HLBM_E_STATE, "coupled motion needs a grid with the lamina");
    if (deform_) return fail(HLBM_E_STATE, "a bending grid takes no coupled motion");
    if (!(m->mass > 0.0) || !(m->stiffness >= 0.0) || !(m->damping >= 0.0) || !(m->y_max > 0.0) ||
        !(std::fabs(m->y0) <= m->y_max) || !(std::fabs(m->v0) < 1.0))
      return fail(HLBM_E_ARG, "invalid coupled-motion parameters");
    if (cfg_.bc != HLBM_BC_PERIODIC &&
        (d_.yc + gey0_ - m->y_max < 1.0 || d_.yc + gey1_ + m->y_max > (double)cfg_.ny - 2.0))
      return fail(HLBM_E_ARG, "grid motion up to y_max leaves the lattice in y");
    HIPCHK(hipStreamSynchronize(s_main_));
    const int64_t cap = std::max<int64_t>(cfg_.max_steps, 1);
    if (!mstate_) HIPCHK(alloc(&mstate_, 2 * (size_t)(cap + 1) * sizeof(double)));
    std::vector<double> st(2 * (size_t)(cap + 1), 0.0);
    st[0] = m->y0;
    st[1] = m->v0;
    HIPCHK(hipMemcpy(mstate_, st.data(), st.size() * sizeof(double), hipMemcpyHostToDevice));
    mot_ = *m;
    fsi_ = true;
    // step 0 at y0 (the previous offset is the current one at k = 0); later
    // steps are written by the device
    StepParams P0 = params_at(0);
    P_host_[0] = P0;
    HIPCHK(hipMemcpy(params_, &P0, sizeof(StepParams), hipMemcpyHostToDevice));
    std::vector<R> uw0(d_.n, (R)m->v0);
    HIPCHK(hipMemcpy(uw_, uw0.data(), uw0.size() * sizeof(R), hipMemcpyHostToDevice));
    // interpolation rows: the rectangle and its position one step earlier
    k2_h_ = P0.iy1 - P0.iy0 + 1 + 3;
    // the two-step band must cover every rectangle |y| <= y_max reaches
    if (two_step_ && !choose_band()) two_step_ = false;
    drop_graphs();
    return HLBM_OK;
  }

  // Prescribed bending of the lamina on a given triangulation (the
  // extension to deformable bodies of Sec. Conclusions). The centreline
  // moves as A sin(omega t) + B sin(omega t + phi) s(x) with s = (2x/b)^2
  // on the lamina; node p of the reference grid sits at local y = y_p +
  // s(x_p) w(y_p) beta_k during step k, beta_k = B sin(omega k + phi),
  // where s falls linearly to 0 from the lamina's ends to the grid's sides
  // and w is 1 across the lamina's thickness and falls linearly to 0 at the
  // grid's top and bottom: the outer boundary moves rigidly, the lamina
  // keeps its thickness. Wall nodes move with the extra velocity
  // B omega cos(omega t + phi) s(x). Each step starts with the geometry
  // update (k_mesh_deform); the refill locates a node's new position in the
  // grid of t_k and takes type 2 inside the bent lamina of t_k.
  static double bend_s(double x, double hb, double ex0, double ex1) {
    if (std::fabs(x) <= hb) return (x / hb) * (x / hb);
    const double side = x < 0.0 ? -ex0 : ex1;
    const double r = 1.0 - (std::fabs(x) - hb) / (side - hb);
    return r > 0.0 ? r : 0.0;
  }
  static double bend_w(double y, double ht, double ey1) {
    if (std::fabs(y) <= ht) return 1.0;
    const double r = 1.0 - (std::fabs(y) - ht) / (ey1 - ht);
    return r > 0.0 ? r : 0.0;
  }

  MeshDeformView<R> deform_view() const {
    MeshDeformView<R> g{};
    g.nnode = grid_.nnode;
    g.ntri = grid_.ntri;
    g.nwall = (int)grid_.wall.size();
    g.x = m_x_;
    g.yref = m_yref_;
    g.prof = m_prof_;
    g.tri = m_tri_;
    g.row = m_row_;
    g.trow = m_trow_;
    g.tlist = m_tlist_;
    g.tslot = m_tslot_;
    g.wall_o = m_wo_;
    g.C = m_C_;
    g.Gx = m_Gx_;
    g.Gy = m_Gy_;
    g.txy = m_txy_;
    g.wall = wall_;
    g.params = params_;
    g.dk = dk_;
    return g;
  }

  int set_deformation(double B, double phi) override {
    if (!has_grid_ || !grid_.mesh) return fail(HLBM_E_UNSUPPORTED, "deformation applies to cases on a given triangulation");
    if (k_ != 0) return fail(HLBM_E_STATE, "the deformation must be set before the first step");
    if (fsi_) return fail(HLBM_E_STATE, "a coupled case does not bend");
    if (!body_) return fail(HLBM_E_STATE, "deformation needs the lamina");
    if (!std::isfinite(B) || !std::isfinite(phi) || !(std::fabs(B) < 1.0))
      return fail(HLBM_E_ARG, "|B| must be finite and below one lattice unit");
    const double hb = 0.5 * grid_.b, ht = 0.5 * grid_.T;
    // the bent lamina stays inside the fictitious rectangle with its donors
    if (!(ht + std::fabs(B) + 1.0 <= gey1_ - kMargin - 1.0))
      return fail(HLBM_E_ARG, "the bent lamina leaves the fictitious rectangle");
    if (!(std::fabs(d_.A * d_.omega) + std::fabs(B * d_.omega) < 1.0))
      return fail(HLBM_E_ARG, "lamina speed must stay below one lattice unit per step");
    const int N = grid_.nnode;
    std::vector<double> prof(N);
    std::vector<R> sx(N);
    for (int p = 0; p < N; ++p) {
      const double sp = bend_s(grid_.x[p], hb, grid_.ex0, grid_.ex1);
      sx[p] = (R)sp;
      prof[p] = sp * bend_w(grid_.y[p], ht, grid_.ey1);
    }
    // a triangle's area is linear in beta: positive at beta = +-B, positive
    // for every configuration
    for (int sgn = -1; sgn <= 1; sgn += 2)
      for (int t = 0; t < grid_.ntri; ++t) {
        double x[3], y[3];
        for (int a = 0; a < 3; ++a) {
          const int n = grid_.tri[3 * t + a];
          x[a] = grid_.x[n];
          y[a] = grid_.y[n] + prof[n] * (sgn * B);
        }
        if (!((x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]) > 0.0))
          return fail(HLBM_E_ARG, "the bent grid folds over (a triangle loses its area)");
      }
    HIPCHK(hipStreamSynchronize(s_main_));
    if (!m_yref_) {
      HIPCHK(upload(&m_yref_, grid_.y.data(), N * sizeof(double)));
      HIPCHK(alloc(&m_prof_, N * sizeof(double)));
      HIPCHK(alloc(&m_sx_, N * sizeof(R)));
      HIPCHK(upload(&m_trow_, grid_.trow.data(), grid_.trow.size() * sizeof(int)));
      HIPCHK(upload(&m_tlist_, grid_.tlist.data(), grid_.tlist.size() * sizeof(int)));
      HIPCHK(upload(&m_tslot_, grid_.tslot.data(), grid_.tslot.size() * sizeof(int)));
      HIPCHK(upload(&m_wo_, grid_.wall_o.data(), std::max<size_t>(1, grid_.wall_o.size()) * sizeof(int)));
      HIPCHK(alloc(&uwb_, std::max<size_t>(1, uw_count()) * sizeof(R)));
    }
    HIPCHK(hipMemcpy(m_prof_, prof.data(), N * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(m_sx_, sx.data(), N * sizeof(R), hipMemcpyHostToDevice));
    dB_ = B;
    dphi_ = phi;
    deform_ = true;
    const int64_t cap = std::max<int64_t>(cfg_.max_steps, 1);
    for (int64_t k = 0; k <= cap; ++k) P_host_[k] = params_at(k);
    HIPCHK(hipMemcpy(params_, P_host_.data(), P_host_.size() * sizeof(StepParams), hipMemcpyHostToDevice));
    std::vector<R> uwb(uw_count());
    for (int64_t k = 0; k < cap; ++k)
      for (int m = 0; m < d_.n; ++m) {
        const double t = (double)k + (double)(m + 1) / (double)d_.n;
        uwb[(size_t)k * d_.n + m] = (R)(dB_ * d_.omega * std::cos(d_.omega * t + dphi_));
      }
    HIPCHK(hipMemcpy(uwb_, uwb.data(), uwb.size() * sizeof(R), hipMemcpyHostToDevice));
    // the configuration of t_0 (stencils and state reads before the first step)
    Kernels<T, R>::mesh_deform(deform_view(), s_main_);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s_main_));
    drop_graphs();
    return HLBM_OK;
  }
  size_t uw_count() const { return (size_t)std::max<int64_t>(cfg_.max_steps, 1) * d_.n; }

  // Capture the graphs of every buffer arrangement the steps will pass
  // through from the current one (the arrangements form a cycle), so that
  // later steps only replay; nothing runs and the state is untouched.
  hipError_t prime_graphs() {
    if (!use_graphs_ || timing_) return hipSuccess;
    void *l0 = lat_[0], *l1 = lat_[1], *l2 = lat_[2];
    const int g0 = gcur_, start = layout_key();
    hipError_t e = hipSuccess;
    for (int i = 0; i < 18 && e == hipSuccess; ++i) {
      hipGraphExec_t ge = nullptr;
      e = graph_for_current_layout(&ge);
      if (e != hipSuccess) break;
      const int key = layout_key();
      lat_[0] = after_graph_[key][0];
      lat_[1] = after_graph_[key][1];
      lat_[2] = after_graph_[key][2];
      gcur_ = after_gcur_[key];
      if (layout_key() == start) break;
    }
    lat_[0] = l0;
    lat_[1] = l1;
    lat_[2] = l2;
    gcur_ = g0;
    return e;
  }

  // captured steps hold the launch shapes they were captured with
  void drop_graphs() {
    for (auto &g : gexec_) {
      if (g) (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  }

  // Time the launch shapes of the stream-collide and the sub-step variants
  // on the current state: every launch reads the current lattice or grid
  // (never written here) and writes the free buffer, which the next step
  // overwrites before reading, so the state is untouched.
  int tune(int trial_steps, hlbm_tuning *t) override {
    if (!t || trial_steps < 0) return fail(HLBM_E_ARG, "invalid tuning request");
    if (trial_steps == 0) {
      const bool keep_shape = t->lattice_threads == 0 && t->lattice_rows == 0;
      if ((!keep_shape && !valid_lattice_shape(*t)) || t->substep_variant < -1 ||
          t->substep_variant >= kSubstepVariantsSingle || t->order < 0 || t->order > 3)
        return fail(HLBM_E_ARG, "invalid schedule");
      if (!keep_shape) {
        lattice_threads_ = t->lattice_threads;
        lattice_rows_ = t->lattice_rows;
      }
      substep_variant_ = t->substep_variant;
      lattice_order_ = t->order & 1;
      two_step_order_ = (t->order >> 1) & 1;
      HIPCHK(hipStreamSynchronize(s_main_));
      drop_graphs();
      HIPCHK(prime_graphs());
      *t = hlbm_tuning{0, lattice_threads_, lattice_rows_, substep_variant_, order_code(), -1, 0, 0, 0.0};
      return HLBM_OK;
    }
    HIPCHK(hipDeviceSynchronize());
    CaseView<T, R> v = view();
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    hipError_t e = hipSuccess;
    // best of two timed passes of `launch` on `st`, in ms
    auto timed = [&](hipStream_t st, auto launch) {
      float best = 3e38f;
      for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {  // the first pass warms up
        e = hipEventRecord(e0, st);
        for (int i = 0; i < trial_steps; ++i) launch();
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0 && ms < best) best = ms;
      }
      return best;
    };
    double total = 0.0;
    float best_ms = 3e38f;
    for (int lt : {128, 256})
      for (int rows : {1, 2, 4})
        for (int ord : {0, 1}) {
          const float ms =
              timed(s_main_, [&] { Kernels<T, R>::stream_collide(v, s_main_, nullptr, nullptr, lt, rows, ord); });
          if (e == hipSuccess && ms < best_ms) {
            best_ms = ms;
            lattice_threads_ = lt;
            lattice_rows_ = rows;
            lattice_order_ = ord;
          }
        }
    if (two_step_) {  // the two-step kernel's tile order (writes B and C, both free between pairs)
      float best2 = 3e38f;
      for (int ord : {0, 1}) {
        const float ms = timed(s_main_, [&] { Kernels<T, R>::stream_collide2(v, s_main_, nullptr, nullptr, ord); });
        if (e == hipSuccess && ms < best2) {
          best2 = ms;
          two_step_order_ = ord;
        }
      }
    }
    total += best_ms;
    if (has_grid_ && grid_.mesh) {  // one sub-step kernel: timed, nothing to choose
      total += timed(s_grid_, [&] {
        for (int m = 0; m < d_.n; ++m)
          Kernels<T, R>::mesh_substep(v, (const R *)gbuf_[gcur_], (R *)gbuf_[1 - gcur_], m, s_grid_);
      });
    } else if (has_grid_) {
      best_ms = 3e38f;
      int best = default_substep_variant<R>();
      for (int sv = 0; sv < kSubstepVariantsSingle; ++sv) {
        const int blk = substep_block(sv);
        const float ms = timed(s_grid_, [&] {
          for (int m = 0; m < d_.n; m += blk)
            Kernels<T, R>::grid_substeps(v, (const R *)gbuf_[gcur_], (R *)gbuf_[1 - gcur_], m,
                                         std::min(blk, d_.n - m), s_grid_, nullptr, nullptr, nullptr, 0, sv);
        });
        if (e == hipSuccess && ms < best_ms) {
          best_ms = ms;
          best = sv;
        }
      }
      substep_variant_ = best;
      total += best_ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(e);
    drop_graphs();
    HIPCHK(prime_graphs());
    *t = hlbm_tuning{0, lattice_threads_, lattice_rows_, substep_variant_, order_code(), -1, 0, 0,
                      total / trial_steps};
    return HLBM_OK;
  }

  int timing_get(int kernel, double *ms, int64_t *count) override {
    if (kernel < 0 || kernel >= kTimedKernels) return fail(HLBM_E_ARG, "unknown kernel id");
    if (ms) *ms = tms_[kernel];
    if (count) *count = tcount_[kernel];
    return HLBM_OK;
  }

  // Reverse mode over all steps taken: windows of ckpt_every steps from the
  // last to the first; each window is recomputed from its checkpoint into the
  // tape, then run backwards step by step.
  int adjoint(const double *dJ, int64_t n, double grad[3]) override {
    if (!dJ || !grad) return fail(HLBM_E_ARG, "null argument");
    if (!has_grid_) return fail(HLBM_E_STATE, "case has no grid, so no force to differentiate");
    if (ckW_ <= 0) return fail(HLBM_E_STATE, "case was created with ckpt_every = 0");
    if (!ck_valid_) return fail(HLBM_E_STATE, "state was replaced after step 0; the checkpoints no longer hold");
    if (fsi_) return fail(HLBM_E_UNSUPPORTED, "adjoint of a case with coupled motion");
    if (n != k_ || n <= 0) return fail(HLBM_E_ARG, "the cotangent must cover every step taken (n = steps)");
    HIPCHK(hipStreamSynchronize(s_main_));
    int rc = adjoint_setup();
    if (rc != HLBM_OK) return rc;
    const size_t lat_r = 9 * plane_ * sizeof(R), grid_r = 9 * (size_t)grid_.nnode * sizeof(R);
    HIPCHK(hipMemsetAsync(alat_[0], 0, lat_r, s_main_));
    HIPCHK(hipMemsetAsync(agrid_[0], 0, grid_r, s_main_));
    HIPCHK(hipMemsetAsync(part_, 0, (size_t)nslots_ * 3 * sizeof(double), s_main_));
    aslot_ = 0;
    if (timing_) HIPCHK(hipEventRecord(tev_adj_[2], s_main_));
    int lc = 0, gc = 0;
    const int64_t nwin = (n + ckW_ - 1) / ckW_;
    auto tape_of = [&](int64_t w) { return (int)(w % ntapes_); };
    auto window = [&](int64_t w, int64_t &k0, int64_t &k1) {
      k0 = w * ckW_;
      k1 = std::min<int64_t>(n, k0 + ckW_);
    };
    // the recompute of window w-1 (stream s_aux_) runs while window w is
    // reversed (s_main_); a tape is rewritten only after its reverse ended
    HIPCHK(hipEventRecord(ev_rev_[0], s_main_));
    HIPCHK(hipEventRecord(ev_rev_[1], s_main_));
    HIPCHK(hipStreamWaitEvent(s_aux_, ev_rev_[0], 0));
    {
      int64_t k0, k1;
      window(nwin - 1, k0, k1);
      COPYCHK(recompute(tape_of(nwin - 1), nwin - 1, k0, k1, s_aux_));
      HIPCHK(hipEventRecord(ev_rec_[tape_of(nwin - 1)], s_aux_));
    }
    for (int64_t w = nwin - 1; w >= 0; --w) {
      const int t = tape_of(w);
      int64_t k0, k1;
      if (w > 0 && ntapes_ == 2) {
        const int tp = tape_of(w - 1);
        window(w - 1, k0, k1);
        HIPCHK(hipStreamWaitEvent(s_aux_, ev_rev_[tp], 0));
        COPYCHK(recompute(tp, w - 1, k0, k1, s_aux_));
        HIPCHK(hipEventRecord(ev_rec_[tp], s_aux_));
      }
      window(w, k0, k1);
      HIPCHK(hipStreamWaitEvent(s_main_, ev_rec_[t], 0));
      for (int64_t k = k1 - 1; k >= k0; --k) HIPCHK(reverse_step(t, k, k0, dJ, lc, gc));
      HIPCHK(hipEventRecord(ev_rev_[t], s_main_));
      if (w > 0 && ntapes_ == 1) {
        window(w - 1, k0, k1);
        HIPCHK(hipStreamWaitEvent(s_aux_, ev_rev_[t], 0));
        COPYCHK(recompute(t, w - 1, k0, k1, s_aux_));
        HIPCHK(hipEventRecord(ev_rec_[t], s_aux_));
      }
    }
    // restore the forward's step counter after the last recompute
    HIPCHK(hipStreamWaitEvent(s_main_, ev_rec_[0], 0));
    if (ntapes_ == 2) HIPCHK(hipStreamWaitEvent(s_main_, ev_rec_[1], 0));
    if (timing_) HIPCHK(harvest_adjoint());
    adj_reduce(part_, nslots_, grad_dev_, s_main_);
    set_step_counter(dk_, k_, s_main_);
    HIPCHK(hipGetLastError());
    if (timing_) HIPCHK(hipEventRecord(tev_adj_[3], s_main_));
    double g[3];
    HIPCHK(hipMemcpyAsync(g, grad_dev_, sizeof(g), hipMemcpyDeviceToHost, s_main_));
    HIPCHK(hipStreamSynchronize(s_main_));
    if (timing_) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, tev_adj_[2], tev_adj_[3]));
      tms_[HLBM_K_ADJOINT] += ms;
      tcount_[HLBM_K_ADJOINT] += n;
    }
    for (int i = 0; i < 3; ++i) grad[i] = g[i];
    adj_lc_ = lc;
    adj_gc_ = gc;
    adj_done_ = true;
    return HLBM_OK;
  }

 private:
  template <class P>
  hipError_t alloc(P **p, size_t bytes) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) {
      owned_.push_back(q);
      owned_bytes_.push_back(bytes);
    }
    *p = (P *)q;
    return e;
  }
  // true when [p, p + n) lies inside one device allocation of this case
  bool owns(const void *p, size_t n) const {
    const char *c = (const char *)p;
    for (size_t i = 0; i < owned_.size(); ++i) {
      const char *a = (const char *)owned_[i];
      if (c >= a && n <= owned_bytes_[i] && (size_t)(c - a) <= owned_bytes_[i] - n) return true;
    }
    return false;
  }
  // an asynchronous copy whose device side (both sides between two device
  // buffers) is checked against this case's allocations before it is enqueued
  hipError_t copy_checked(void *dst, const void *src, size_t n, hipMemcpyKind kind, hipStream_t st) {
    const bool dev_dst = kind == hipMemcpyDeviceToDevice || kind == hipMemcpyHostToDevice;
    const bool dev_src = kind == hipMemcpyDeviceToDevice || kind == hipMemcpyDeviceToHost;
    if ((dev_dst && !owns(dst, n)) || (dev_src && !owns(src, n))) {
      copy_fault_ = true;
      return hipErrorInvalidValue;
    }
    return hipMemcpyAsync(dst, src, n, kind, st);
  }
  template <class P>
  hipError_t upload(P **p, const void *src, size_t bytes) {
    hipError_t e = alloc(p, bytes);
    if (e == hipSuccess && bytes && src) e = hipMemcpy((void *)*p, src, bytes, hipMemcpyHostToDevice);
    return e;
  }
  void release() {
    if (s_aux_) (void)hipStreamSynchronize(s_aux_);
    if (s_main_) (void)hipStreamSynchronize(s_main_);
    if (s_grid_ && s_grid_ != s_main_) (void)hipStreamSynchronize(s_grid_);
    for (auto &g : gexec_)
      if (g) (void)hipGraphExecDestroy(g);
    for (void *p : owned_) (void)hipFree(p);
    owned_.clear();
    for (auto &ring : tev_)
      for (auto &e : ring)
        if (e) (void)hipEventDestroy(e);
    for (auto &ring : tev3_)
      for (auto &e : ring)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : tev_adj_)
      if (e) (void)hipEventDestroy(e);
    for (auto &pr : tev_adj_ring_)
      for (auto &e : pr)
        if (e) (void)hipEventDestroy(e);
    if (ev_fork_) (void)hipEventDestroy(ev_fork_);
    if (ev_join_) (void)hipEventDestroy(ev_join_);
    if (ev_flag_) (void)hipEventDestroy(ev_flag_);
    if (hflag_) (void)hipHostFree(hflag_);
    hflag_ = nullptr;
    for (auto &e : ev_rec_)
      if (e) (void)hipEventDestroy(e);
    for (auto &e : ev_rev_)
      if (e) (void)hipEventDestroy(e);
    if (s_aux_) (void)hipStreamDestroy(s_aux_);
    if (s_grid_ && s_grid_ != s_main_) (void)hipStreamDestroy(s_grid_);
    if (s_main_) (void)hipStreamDestroy(s_main_);
  }
  int fail(int code, const char *msg) {
    err = msg;
    return code;
  }

  double motion(int64_t k) const {
    if (fsi_) return k == 0 ? mot_.y0 : 0.0;  // coupled: only t_0 is known on the host
    return d_.A * std::sin(d_.omega * (double)k);
  }

  // Fictitious rectangle: the grid's node bounding box at offset y, inset by
  // two lattice units; lattice node (i, j) is inside when the closed
  // rectangle holds it, i.e. ceil(x0) <= i <= floor(x1), same in y.
  void rect(double y, int &ix0, int &ix1, int &iy0, int &iy1) const {
    const double rx0 = d_.xc + gex0_ + kMargin;
    const double rx1 = d_.xc + gex1_ - kMargin;
    const double ry0 = d_.yc + y + gey0_ + kMargin;
    const double ry1 = d_.yc + y + gey1_ - kMargin;
    ix0 = (int)std::ceil(rx0);
    ix1 = (int)std::floor(rx1);
    iy0 = (int)std::ceil(ry0);
    iy1 = (int)std::floor(ry1);
  }

  // Band of the two-step path: every lattice node within kBand of a
  // fictitious rectangle of any step (k = 0 .. max_steps, and k - 1 = 0),
  // so a node outside it meets no interpolation node, carried node, grid
  // donor or refill donor in either step of a pair. False when the path
  // does not apply (lattice too small for its tile, ring boundaries, or a
  // band that would wrap across a periodic edge).
  bool choose_band() {
    if (cfg_.bc != HLBM_BC_PERIODIC_X_WALLS_Y && cfg_.bc != HLBM_BC_PERIODIC && cfg_.bc != HLBM_BC_PAPER) return false;
    if (cfg_.nx < kTwoStepTX + 2 || cfg_.ny < kTwoStepTY + 2) return false;
    if (!has_grid_) return true;  // no band: every node takes both steps at once
    constexpr int kBand = 6;
    int x0 = cfg_.nx, x1 = -1, y0 = cfg_.ny, y1 = -1;
    for (const StepParams &P : P_host_) {
      x0 = std::min({x0, P.ix0, P.pix0});
      x1 = std::max({x1, P.ix1, P.pix1});
      y0 = std::min({y0, P.iy0, P.piy0});
      y1 = std::max({y1, P.iy1, P.piy1});
    }
    if (fsi_) {  // every offset |y| <= y_max
      for (double y : {-mot_.y_max, mot_.y_max}) {
        int a, b, c, d;
        rect(y, a, b, c, d);
        y0 = std::min(y0, c);
        y1 = std::max(y1, d);
      }
    }
    x0 -= kBand;
    x1 += kBand;
    y0 -= kBand;
    y1 += kBand;
    if (x0 < 0 || y0 < 0 || x1 >= cfg_.nx || y1 >= cfg_.ny) return false;
    band_[0] = x0;
    band_[1] = x1;
    band_[2] = y0;
    band_[3] = y1;
    return true;
  }

  StepParams params_at(int64_t k) const {
    StepParams P;
    P.y = motion(k);
    P.y1 = motion(k + 1);
    const double yp = k > 0 ? motion(k - 1) : P.y;
    P.ybase = d_.yc + P.y;
    P.ybase1 = d_.yc + P.y1;
    rect(P.y, P.ix0, P.ix1, P.iy0, P.iy1);
    rect(yp, P.pix0, P.pix1, P.piy0, P.piy1);
    P.beta = deform_ ? dB_ * std::sin(d_.omega * (double)k + dphi_) : 0.0;
    P.beta1 = deform_ ? dB_ * std::sin(d_.omega * (double)(k + 1) + dphi_) : 0.0;
    return P;
  }

  CaseView<T, R> view() const {
    CaseView<T, R> v{};
    v.flag = flag_;
    v.A = (const T *)lat_[0];
    v.B = (T *)lat_[1];
    v.C = (T *)lat_[2];
    v.nx = cfg_.nx;
    v.plane = plane_;
    v.ny = cfg_.ny;
    v.wx0 = 0;
    v.wy0 = 0;
    v.ww = cfg_.nx;
    v.wh = cfg_.ny;
    v.bx0 = band_[0];
    v.bx1 = band_[1];
    v.by0 = band_[2];
    v.by1 = band_[3];
    if (fsi_) {
      v.mot.on = 1;
      v.mot.M = mot_.mass;
      v.mot.K = mot_.stiffness;
      v.mot.C = mot_.damping;
      v.mot.y_max = mot_.y_max;
      v.mot.yc = d_.yc;
      v.mot.c0 = gey0_;
      v.mot.c1 = gey1_;
      v.mot.margin = kMargin;
      v.mot.state = mstate_;
      v.mot.cap = cfg_.max_steps;
    }
    v.bc = cfg_.bc;
    v.inv_tau = (R)(1.0 / cfg_.tau);
    v.g_post = (R)(2.0 * (cfg_.tau - 1.0) / (2.0 * cfg_.tau - 1.0));
    v.k_neq = (R)(1.0 - 1.0 / (2.0 * cfg_.tau));
    v.has_grid = has_grid_;
    if (has_grid_) {
      v.nux = cfg_.nux;
      v.nuy = cfg_.nuy;
      v.nnode = grid_.nnode;
      v.n_iface = (int)grid_.iface.size();
      v.n_wall_edges = (int)grid_.wall.size();
      v.n_sub = d_.n;
      v.h = h_;
      v.xc = d_.xc;
      v.yc = d_.yc;
      v.half_b = 0.5 * grid_.b;
      v.half_T = 0.5 * grid_.T;
      v.body = body_;
      v.gx = dgx_;
      v.gy = dgy_;
      v.ncode = ncode_;
      v.tab = tab_;
      v.iface = iface_;
      if (grid_.mesh) {
        v.mesh = 1;
        v.nux = v.nuy = 0;
        v.m_row = m_row_;
        v.m_col = m_col_;
        v.m_C = m_C_;
        v.m_Gx = m_Gx_;
        v.m_Gy = m_Gy_;
        v.m_x = m_x_;
        v.m_y = m_y_;
        v.m_type = m_type_;
        v.mg = MeshGeom{m_tri_, m_txy_, m_bstart_, m_blist_, grid_.bx0, grid_.by0, grid_.bnx, grid_.bny};
        if (deform_) {
          v.deform = 1;
          v.m_yref = m_yref_;
          v.m_prof = m_prof_;
          v.m_sx = m_sx_;
          v.uwb = uwb_;
        }
      }
      v.wall = wall_;
      v.star_f = star_f_;
      v.star_n = star_n_;
      v.dt_u = (R)(1.0 / (double)d_.n);
      v.dt_over_tau_u = (R)((1.0 / (double)d_.n) / d_.tau_u);
      v.uw = uw_;
      v.params = params_;
      v.dk = dk_;
      v.dkl = dk_;
      v.hist = hist_;
      v.counts = counts_;
      v.k2_x0 = k2_x0_;
      v.k2_w = k2_w_;
      v.k2_h = k2_h_;
    }
    v.lat[0] = (T *)lat_base_;
    v.lat[1] = (T *)(lat_base_ == lat_[0] ? lat_[1] : lat_[0]);
    v.grid[0] = (R *)gbuf_[0];
    v.grid[1] = (R *)gbuf_[1];
    v.max_steps = cfg_.max_steps;
    return v;
  }

 public:
  // ---- hooks for a batch that advances this case with case-batched kernels
  CaseView<T, R> batched_view() const { return view(); }
  int64_t steps_taken() const { return k_; }
  int64_t max_steps() const { return cfg_.max_steps; }
  int n_sub() const { return d_.n; }
  int64_t *step_counter() const { return dk_; }
  int *flag() const { return flag_; }
  // host bookkeeping after m steps done on the device by batched kernels
  void advance_host(int64_t m) {
    const int blk = substep_block(substep_variant_);
    const int launches = (d_.n + blk - 1) / blk;
    if (m & 1) {
      std::swap(lat_[0], lat_[1]);
      if ((launches + 1) & 1) gcur_ = 1 - gcur_;
    }
    k_ += m;
  }
  // ---- hooks for a multi-level handle that runs this case as its finest level
  hipStream_t stream() const { return s_main_; }
  void *lattice_buffer(int i) const { return lat_[i]; }  // 0: state at t_k, 1: at t_{k-1}
  size_t plane() const { return plane_; }
  bool has_grid() const { return has_grid_; }
  hipError_t enqueue_one() { return enqueue_step(); }
  struct Layout {
    void *l0, *l1, *l2;
    int gcur;
    int64_t k;
  };
  Layout layout() const { return {lat_[0], lat_[1], lat_[2], gcur_, k_}; }
  void set_layout(const Layout &l) {
    lat_[0] = l.l0;
    lat_[1] = l.l1;
    lat_[2] = l.l2;
    gcur_ = l.gcur;
    k_ = l.k;
  }
  // every lattice and grid buffer, for snapshots
  void buffers(void **lat, void **grid, size_t *lat_bytes, size_t *grid_bytes) const {
    lat[0] = lat_[0];
    lat[1] = lat_[1];
    grid[0] = gbuf_[0];
    grid[1] = gbuf_[1];
    *lat_bytes = 9 * plane_ * sizeof(T);
    *grid_bytes = has_grid_ ? 9 * (size_t)grid_.nnode * sizeof(R) : 0;
  }
  unsigned long long *refill_counters() const { return counts_; }
  int64_t lattice_nodes() const { return (int64_t)nodes_; }
  int64_t grid_nodes() const { return has_grid_ ? grid_.nnode : 0; }

 private:

  hipError_t harvest_adjoint() {
    if (aslot_ == 0) return hipSuccess;
    hipError_t e = hipEventSynchronize(tev_adj_ring_[aslot_ - 1][1]);
    if (e != hipSuccess) return e;
    for (int i = 0; i < aslot_; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, tev_adj_ring_[i][0], tev_adj_ring_[i][1]) == hipSuccess) {
        tms_[HLBM_K_ADJ_STREAM_COLLIDE] += ms;
        tcount_[HLBM_K_ADJ_STREAM_COLLIDE] += 1;
      }
      if (has_grid_ && hipEventElapsedTime(&ms, tev_adj_ring_[i][2], tev_adj_ring_[i][3]) == hipSuccess) {
        tms_[HLBM_K_ADJ_SUBSTEPS] += ms;
        tcount_[HLBM_K_ADJ_SUBSTEPS] += 1;
      }
    }
    aslot_ = 0;
    return hipSuccess;
  }

  // Accumulates the timings of the steps recorded in the event ring (the
  // steps ran back to back; only here does the host wait for them).
  hipError_t harvest() {
    hipError_t e = timing_ == 3 ? hipSuccess : hipEventSynchronize(tev_[tslot_ - 1][2]);
    if (e == hipSuccess) e = hipStreamSynchronize(s_main_);
    if (e == hipSuccess && s_grid_ != s_main_) e = hipStreamSynchronize(s_grid_);
    if (e != hipSuccess) return e;
    for (int i = 0; i < tslot_; ++i) {
      hipEvent_t *t = tev_[i];
      auto add = [&](int id, hipEvent_t a, hipEvent_t b) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, a, b) == hipSuccess) {
          tms_[id] += ms;
          tcount_[id] += 1;
        }
      };
      if (timing_ == 3) {
        for (int j = 0; j < sub_n_[i]; ++j) add(HLBM_K_SUBSTEP_LAUNCH, tev3_[i][2 * j], tev3_[i][2 * j + 1]);
        sub_n_[i] = 0;
        continue;
      }
      add(HLBM_K_STREAM_COLLIDE, t[8], t[2]);
      if (timing_ != 1) continue;
      if (has_grid_) {
        add(HLBM_K_LATTICE_FROM_GRID, t[0], t[1]);
        add(HLBM_K_GRID_SUBSTEPS, t[3], t[4]);
        add(HLBM_K_REFILL, t[4], t[5]);
        add(HLBM_K_FORCE, t[5], t[6]);
      }
      add(HLBM_K_STEP, t[0], t[7]);
    }
    tslot_ = 0;
    return hipSuccess;
  }

  // ---- adjoint workspace ------------------------------------------------------
  size_t tape_grid_elems() const { return 9 * (size_t)grid_.nnode; }
  T *tape_lat(int t, int64_t j) const { return (T *)tape_lat_[t] + (size_t)j * 9 * plane_; }
  R *tape_grid(int t, int64_t j, int m) const {
    return tape_grid_[t] + ((size_t)j * (d_.n + 1) + m) * tape_grid_elems();
  }
  R *tape_wall(int t, int64_t j) const { return wtape_[t] + (size_t)j * d_.n * 3 * std::max(n_wall_, 1); }

  // Allocates the tape and the adjoint buffers on first use and fills the
  // step-independent part of the kernels' context.
  int adjoint_setup() {
    if (adj_ready_) return HLBM_OK;
    const int N = grid_.nnode;
    // lattice rows and columns that can be bilinear donors: the grid's
    // bounding box over the whole motion, one node wider
    // (graded: the first and last column and row of the given spacing)
    const bool graded = !gx_.empty();
    const double hx0 = graded ? gx_.front() : (double)(0 - cfg_.nux / 2) * h_;
    const double hx1 = graded ? gx_.back() : (double)(cfg_.nux - 1 - cfg_.nux / 2) * h_;
    const double hy = graded ? std::max(-gy_.front(), gy_.back()) : 0.5 * (double)(cfg_.nuy - 1) * h_;
    double ymin = 1e300, ymax = -1e300;
    for (const StepParams &P : P_host_) {
      ymin = std::min(ymin, std::min(P.ybase, P.ybase1));
      ymax = std::max(ymax, std::max(P.ybase, P.ybase1));
    }
    ex0_ = (int)std::floor(d_.xc + hx0);
    ew_ = (int)std::floor(d_.xc + hx1) + 2 - ex0_;
    ey0_ = (int)std::floor(ymin - hy);
    eh_ = (int)std::floor(ymax + hy) + 2 - ey0_;
    if (ex0_ < 0 || ex0_ + ew_ > cfg_.nx || ey0_ < 0 || ey0_ + eh_ > cfg_.ny)
      return fail(HLBM_E_UNSUPPORTED, "lattice donors of the grid wrap across a periodic boundary");
    const size_t tape_lat_bytes = (size_t)(ckW_ + 1) * 9 * plane_ * sizeof(T);
    const size_t tape_grid_bytes = ((size_t)ckW_ * (d_.n + 1) + 1) * tape_grid_elems() * sizeof(R);
    size_t free_b = 0, total_b = 0;
    HIPCHK(hipMemGetInfo(&free_b, &total_b));
    n_wall_ = (int)std::count(grid_.type.begin(), grid_.type.end(), (int)NODE_WALL);
    const size_t tape_wall_bytes = (size_t)ckW_ * d_.n * 3 * std::max(n_wall_, 1) * sizeof(R);
    const size_t one = tape_lat_bytes + tape_grid_bytes + tape_wall_bytes;
    const size_t fixed = 2 * 9 * plane_ * sizeof(R) + ((size_t)256 << 20);
    // two tapes let the recompute of the previous window run on a second
    // stream while this window is reversed; one tape runs them in turn
    if (one + fixed > free_b) return fail(HLBM_E_NOMEM, "adjoint tape does not fit in device memory: use a smaller ckpt_every");
    ntapes_ = (2 * one + fixed <= free_b && !std::getenv("HLBM_ONE_TAPE")) ? 2 : 1;
    for (int t = 0; t < ntapes_; ++t) {
      HIPCHK(alloc(&tape_lat_[t], tape_lat_bytes));
      HIPCHK(alloc(&tape_grid_[t], tape_grid_bytes));
      HIPCHK(alloc(&wtape_[t], tape_wall_bytes));
    }
    HIPCHK(alloc(&astar_f_, 9 * (size_t)N * sizeof(R)));
    HIPCHK(alloc(&astar_n_, 9 * (size_t)N * sizeof(R)));
    HIPCHK(hipStreamCreateWithFlags(&s_aux_, hipStreamNonBlocking));
    for (int t = 0; t < 2; ++t) {
      HIPCHK(hipEventCreateWithFlags(&ev_rec_[t], hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&ev_rev_[t], hipEventDisableTiming));
    }
    for (int i = 0; i < 2; ++i) {
      HIPCHK(alloc(&alat_[i], 9 * plane_ * sizeof(R)));
      HIPCHK(alloc(&agrid_[i], 9 * (size_t)N * sizeof(R)));
    }
    HIPCHK(alloc(&M2_, 3 * (size_t)N * sizeof(R)));
    HIPCHK(alloc(&sbf_, 9 * (size_t)N * sizeof(R)));
    HIPCHK(alloc(&sbn_, 9 * (size_t)N * sizeof(R)));
    HIPCHK(alloc(&Z1_, 12 * (size_t)N * sizeof(R)));
    HIPCHK(alloc(&Z2_, 12 * (size_t)N * sizeof(R)));
    HIPCHK(alloc(&zf_, (size_t)N));
    HIPCHK(alloc(&Z3_, 12 * (size_t)k2_w_ * k2_h_ * sizeof(R)));
    HIPCHK(alloc(&E_, 9 * (size_t)ew_ * eh_ * sizeof(R)));
    if (cfg_.bc == HLBM_BC_PAPER) HIPCHK(alloc(&Vend_, 4 * 9 * (size_t)cfg_.nx * sizeof(R)));
    HIPCHK(alloc(&grad_dev_, 3 * sizeof(double)));
    HIPCHK(alloc(&counts_scratch_, 2 * sizeof(unsigned long long)));
    HIPCHK(hipMemset(Z2_, 0, 12 * (size_t)N * sizeof(R)));
    // wall nodes and, per node, the sum over its wall edges of (len/2) n
    std::vector<int> wn;
    std::vector<double> nrm(2 * (size_t)N, 0.0);
    for (int p = 0; p < N; ++p)
      if (grid_.type[p] == NODE_WALL) wn.push_back(p);
    for (const WallEdge &e : grid_.wall)
      for (int s = 0; s < 2; ++s) {
        const int p = s ? e.b : e.a;
        nrm[p] += 0.5 * e.len * e.nx;
        nrm[N + p] += 0.5 * e.len * e.ny;
      }
    HIPCHK(upload(&wall_nodes_, wn.data(), wn.size() * sizeof(int)));
    HIPCHK(upload(&wall_nrm_, nrm.data(), nrm.size() * sizeof(double)));
    std::vector<int> widx(N, -1);
    for (size_t w = 0; w < wn.size(); ++w) widx[wn[w]] = (int)w;
    std::vector<unsigned char> ntype(N);
    for (int p = 0; p < N; ++p) ntype[p] = (unsigned char)grid_.type[p];
    HIPCHK(upload(&widx_, widx.data(), widx.size() * sizeof(int)));
    HIPCHK(upload(&ntype_, ntype.data(), ntype.size()));
    n_wall_ = (int)wn.size();
    // transposed stencils: slot s of node q holds what its neighbour at slot
    // s applies to q (the neighbour's slot 8 - s), deduplicated into classes
    {
      std::vector<AdjClass<double>> atab;
      std::vector<int> acls(N);
      std::map<std::string, int> seen;
      for (int q = 0; q < N; ++q) {
        const int i = q % cfg_.nux, j = q / cfg_.nux;
        AdjClass<double> a;
        std::memset(&a, 0, sizeof(a));
        a.type = grid_.type[q];
        for (int s = 0; s < NSLOT; ++s) {
          const int ii = i + s % 3 - 1, jj = j + s / 3 - 1;
          if (ii < 0 || jj < 0 || ii >= cfg_.nux || jj >= cfg_.nuy) continue;
          const int p = jj * cfg_.nux + ii;
          const GridClass<double> &cp = grid_.classes[grid_.cls[p]];
          a.Gx[s] = cp.Gx[NSLOT - 1 - s];
          a.Gy[s] = cp.Gy[NSLOT - 1 - s];
          a.C[s] = cp.C[NSLOT - 1 - s];
          if (grid_.type[p] == NODE_INTERFACE && grid_.type[q] == NODE_INTERFACE) a.star |= 1 << s;
        }
        const std::string key((const char *)&a, sizeof(a));
        auto it = seen.find(key);
        if (it == seen.end()) {
          it = seen.emplace(key, (int)atab.size()).first;
          atab.push_back(a);
        }
        acls[q] = it->second;
      }
      std::vector<AdjClass<R>> at(atab.size());
      for (size_t k = 0; k < atab.size(); ++k) {
        std::memset(&at[k], 0, sizeof(at[k]));
        for (int s = 0; s < NSLOT; ++s) {
          at[k].Gx[s] = (R)atab[k].Gx[s];
          at[k].Gy[s] = (R)atab[k].Gy[s];
          at[k].C[s] = (R)atab[k].C[s];
        }
        at[k].star = atab[k].star;
        at[k].type = atab[k].type;
      }
      HIPCHK(upload(&atab_, at.data(), at.size() * sizeof(AdjClass<R>)));
      // per node: 4 class + the diagonal slot pairs its class lacks (bit 0:
      // slots 2 and 6, bit 1: slots 0 and 8), which a wave may skip
      for (int q = 0; q < N; ++q) {
        const AdjClass<R> &a = at[acls[q]];
        auto zero = [&](int s) { return a.C[s] == R(0) && a.Gx[s] == R(0) && a.Gy[s] == R(0); };
        acls[q] = 4 * acls[q] + (zero(2) && zero(6) ? 1 : 0) + (zero(0) && zero(8) ? 2 : 0);
      }
      HIPCHK(upload(&acls_, acls.data(), acls.size() * sizeof(int)));
      n_adj_classes_ = (int)at.size();
    }
    AdjCtx<T, R> &c = actx_;
    std::memset(&c, 0, sizeof(c));
    c.nx = cfg_.nx;
    c.plane = plane_;
    c.ny = cfg_.ny;
    c.bc = cfg_.bc;
    c.has_grid = 1;
    c.tau = cfg_.tau;
    c.tau_u = d_.tau_u;
    const CaseView<T, R> v = view();
    c.inv_tau = v.inv_tau;
    c.g_post = v.g_post;
    c.k_neq = v.k_neq;
    c.dt = v.dt_u;
    c.dt_tau = v.dt_over_tau_u;
    c.gg = dev::GridGeom{cfg_.nux, cfg_.nuy, h_, d_.xc, v.half_b, v.half_T, (int)body_, v.gx, v.gy};
    c.nnode = N;
    c.n_iface = (int)grid_.iface.size();
    c.n_wall = (int)wn.size();
    c.ncode = ncode_;
    c.tab = tab_;
    c.iface = iface_;
    c.wall_nodes = wall_nodes_;
    c.widx = widx_;
    c.ntype = ntype_;
    c.acls = acls_;
    c.atab = atab_;
    c.wall_nrm = wall_nrm_;
    c.star_f = astar_f_;
    c.star_n = astar_n_;
    c.M2 = M2_;
    c.sbf = sbf_;
    c.sbn = sbn_;
    c.Z1 = Z1_;
    c.Z2 = Z2_;
    c.zf = zf_;
    c.Z3 = Z3_;
    c.k2_x0 = k2_x0_;
    c.k2_w = k2_w_;
    c.k2_h = k2_h_;
    c.E = E_;
    c.Vend = Vend_;
    c.ex0 = ex0_;
    c.ey0 = ey0_;
    c.ew = ew_;
    c.eh = eh_;
    using AK = AdjKernels<T, R>;
    slot_refill_ = 0;
    slot_sub_ = slot_refill_ + AK::refill_slots(c);
    slot_eg_ = slot_sub_ + AK::substep_slots(c);
    slot_sc_ = slot_eg_ + AK::donor_gather_slots(c);
    slot_fg_ = slot_sc_ + AK::stream_collide_slots(c);
    slot_fgg_ = slot_fg_ + AK::from_grid_slots(c);
    nslots_ = slot_fgg_ + AK::from_grid_gather_slots(c);
    HIPCHK(alloc(&part_, (size_t)nslots_ * 3 * sizeof(double)));
    c.part = part_;
    for (auto &e : tev_adj_)
      if (!e) HIPCHK(hipEventCreate(&e));
    for (auto &pr : tev_adj_ring_)
      for (auto &e : pr)
        if (!e) HIPCHK(hipEventCreate(&e));
    adj_ready_ = true;
    return HLBM_OK;
  }

  // Forward steps k0 .. k1-1 from checkpoint w into tape t on stream st,
  // keeping every lattice after its grid-to-lattice writes, every grid state
  // of every sub-step and the wall moments the adjoint needs.
  hipError_t recompute(int t, int64_t w, int64_t k0, int64_t k1, hipStream_t st) {
    if (t < 0 || t >= ntapes_ || w < 0 || w >= nck_ || k1 - k0 > ckW_) return hipErrorInvalidValue;
    hipError_t e = copy_checked(tape_lat(t, 0), (char *)ck_lat_ + (size_t)w * ck_lat_bytes_, ck_lat_bytes_,
                                hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    e = copy_checked(tape_grid(t, 0, 0), (char *)ck_grid_ + (size_t)w * ck_grid_bytes_, ck_grid_bytes_,
                     hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    for (int64_t k = k0; k < k1; ++k) {
      const int64_t j = k - k0;
      set_step_counter(dk_, k, st);
      CaseView<T, R> v = view();
      v.A = tape_lat(t, j);
      v.B = tape_lat(t, j + 1);
      v.counts = counts_scratch_;
      Kernels<T, R>::lattice_from_grid(v, tape_grid(t, j, 0), st);
      // (the stream-collide launch also computes the interface donors)
      Kernels<T, R>::stream_collide(v, st, nullptr, nullptr, lattice_threads_, lattice_rows_, lattice_order_, true);
      for (int m = 0; m < d_.n; m += kSubstepBlock) {
        const int cnt = std::min(kSubstepBlock, d_.n - m);
        // the tape is written in blocks of kSubstepBlock sub-steps
        const int sv = substep_block(substep_variant_) == kSubstepBlock ? substep_variant_ : -1;
        Kernels<T, R>::grid_substeps(v, tape_grid(t, j, m), tape_grid(t, j, m + cnt), m, cnt, st, tape_grid(t, j, 0),
                                     tape_wall(t, j), widx_, std::max(n_wall_, 1), sv);
      }
      Kernels<T, R>::refill(v, tape_grid(t, j, d_.n), tape_grid(t, j + 1, 0), st);
    }
    return hipGetLastError();
  }

  // One structured step backwards: (alat_[lc], agrid_[gc]) hold the adjoints
  // of the lattice and grid at t_{k+1} on entry and of those at t_k on exit.
  hipError_t reverse_step(int tape, int64_t k, int64_t k0, const double *dJ, int &lc, int &gc) {
    using AK = AdjKernels<T, R>;
    const int64_t j = k - k0;
    if (tape < 0 || tape >= ntapes_ || j < 0 || j >= ckW_) return hipErrorInvalidValue;
    AdjCtx<T, R> c = actx_;
    c.Lt = tape_lat(tape, j);
    c.Lb_next = alat_[lc];
    c.Lb = alat_[1 - lc];
    c.P = P_host_[k];
    const double A = d_.A, om = d_.omega;
    c.dyA = std::sin(om * (double)k);
    c.dyW = A * (double)k * std::cos(om * (double)k);
    c.dyA1 = std::sin(om * (double)(k + 1));
    c.dyW1 = A * (double)(k + 1) * std::cos(om * (double)(k + 1));
    c.wfx = dJ[2 * k];
    c.wfy = dJ[2 * k + 1];
    c.U0 = tape_grid(tape, j, 0);
    c.Un = tape_grid(tape, j, d_.n);
    c.wt = tape_wall(tape, j);
    c.Ub_next = agrid_[gc];
    c.Ubn = agrid_[1 - gc];
    AK::star_refill(c, slot_refill_, s_main_);
    int gin = 1 - gc;  // holds the adjoint of the grid after sub-step m_hi + 1
    for (int m_hi = d_.n - 1; m_hi >= 0; m_hi -= 4) {
      const int count = std::min(4, m_hi + 1);
      AdjSubScal<R> sc{};
      for (int i = 0; i < count; ++i) {
        const double tm = (double)k + (double)(m_hi - i + 1) / (double)d_.n;
        sc.uw[i] = (R)(A * om * std::cos(om * tm));
        sc.duwA[i] = om * std::cos(om * tm);
        sc.duwW[i] = A * std::cos(om * tm) - A * om * tm * std::sin(om * tm);
      }
      const bool timed = timing_ && m_hi == d_.n - 1;  // the step's first reverse launch
      AK::substeps(c, tape_grid(tape, j, 0), agrid_[gin], agrid_[1 - gin], m_hi, count, sc, m_hi == d_.n - 1,
                   m_hi - count + 1 == 0, slot_sub_, s_main_, timed ? tev_adj_ring_[aslot_][2] : nullptr,
                   timed ? tev_adj_ring_[aslot_][3] : nullptr);
      gin = 1 - gin;
    }
    AK::donor_gather(c, slot_eg_, s_main_);
    if (timing_) {
      AK::stream_collide(c, slot_sc_, s_main_, tev_adj_ring_[aslot_][0], tev_adj_ring_[aslot_][1]);
    } else {
      AK::stream_collide(c, slot_sc_, s_main_);
    }
    AK::from_grid(c, slot_fg_, s_main_);
    AK::from_grid_gather(c, agrid_[gin], slot_fgg_, s_main_);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (timing_ && ++aslot_ == kTimingRing) {
      e = harvest_adjoint();
      if (e != hipSuccess) return e;
    }
    lc = 1 - lc;
    gc = gin;
    return hipSuccess;
  }

  hlbm_config cfg_{};
  Derived d_{};
  double h_ = 1.0;
  bool has_grid_ = false, body_ = false;
  size_t nodes_ = 0;  // lattice nodes nx * ny
  size_t plane_ = 0;  // population-plane stride of every lattice-shaped device array
  HostGrid grid_;
  int dev_ = 0;  // the device the case was created on
  hipStream_t s_main_ = nullptr, s_grid_ = nullptr;
  hipEvent_t ev_fork_ = nullptr, ev_join_ = nullptr;
  static constexpr int kTimingRing = 64;  // steps recorded between harvests
  hipEvent_t tev_[kTimingRing][9] = {};
  // level 3: start and end events of each sub-step launch of a step
  static constexpr int kTimedLaunches = 16;
  hipEvent_t tev3_[kTimingRing][2 * kTimedLaunches] = {};
  int sub_n_[kTimingRing] = {};
  int tslot_ = 0;
  int timing_ = 0;  // 1: every kernel, 2: the stream-collide only
  int substep_variant_ = -1;  // grid sub-step kernel variant (-1: the default for R)
  int lattice_threads_ = kLatticeThreads, lattice_rows_ = kLatticeRows;  // stream-collide launch shape
  int lattice_order_ = 0;  // 1: stream-collide rows banded by XCD
  int two_step_order_ = 1;  // 1: two-step tiles in staggered runs per XCD (0: in turn)
  int order_code() const { return lattice_order_ | (two_step_order_ << 1); }
  static constexpr int kTimedKernels = 10;  // HLBM_K_* ids
  double tms_[kTimedKernels] = {};
  int64_t tcount_[kTimedKernels] = {};
  int sub_mark_ = -1;  // timing slot whose first sub-step launch is timed (level 3)
  std::vector<void *> owned_;
  std::vector<size_t> owned_bytes_;  // requested bytes of each owned_ entry
  bool copy_fault_ = false;          // a copy was refused for leaving its allocation
  void *lat_[3] = {nullptr, nullptr, nullptr};  // state at t_k, free, free (two-step path)
  void *phys_[3] = {nullptr, nullptr, nullptr};  // the physical buffers
  bool two_step_ = false;
  bool fsi_ = false;  // two-way coupled motion (hlbm_set_motion)
  double gex0_ = 0.0, gex1_ = 0.0, gey0_ = 0.0, gey1_ = 0.0;  // local extents of the grid
  std::vector<double> gx_, gy_;  // graded grid: columns and rows (empty: uniform)
  double *dgx_ = nullptr, *dgy_ = nullptr;
  hlbm_motion mot_{};
  double *mstate_ = nullptr;  // [max_steps + 1][2] (y, v) on the device
  int band_[4] = {-10, -20, -10, -20};  // x0, x1, y0, y1 of the band (inclusive; empty, far outside)
  void *after_graph_[18][3] = {};
  int after_gcur_[18] = {};
  void *gbuf_[2] = {nullptr, nullptr};
  int gcur_ = 0;
  R *star_f_ = nullptr, *star_n_ = nullptr;
  GridClass<R> *tab_ = nullptr;
  int *ncode_ = nullptr, *iface_ = nullptr;
  // unstructured grid (device copies of the HostGrid mesh fields)
  int *m_row_ = nullptr, *m_col_ = nullptr, *m_type_ = nullptr, *m_tri_ = nullptr;
  int *m_bstart_ = nullptr, *m_blist_ = nullptr;
  R *m_C_ = nullptr, *m_Gx_ = nullptr, *m_Gy_ = nullptr;
  double *m_x_ = nullptr, *m_y_ = nullptr, *m_txy_ = nullptr;
  WallEdge *wall_ = nullptr;
  // prescribed bending of an unstructured grid (hlbm_set_deformation)
  bool deform_ = false;
  double dB_ = 0.0, dphi_ = 0.0;
  double *m_yref_ = nullptr, *m_prof_ = nullptr;
  R *m_sx_ = nullptr, *uwb_ = nullptr;
  int *m_trow_ = nullptr, *m_tlist_ = nullptr, *m_tslot_ = nullptr, *m_wo_ = nullptr;
  StepParams *params_ = nullptr;
  R *uw_ = nullptr;
  double *hist_ = nullptr;
  int64_t *dk_ = nullptr;
  int *flag_ = nullptr;
  int *hflag_ = nullptr;          // pinned: the flag as last copied by step_async
  hipEvent_t ev_flag_ = nullptr;  // recorded after that copy
  bool flag_copied_ = false;      // a copy has been enqueued
  bool pending_ = false;          // steps enqueued by step_async not yet waited for
  unsigned long long *counts_ = nullptr;
  unsigned *done_ = nullptr;  // workgroups done in the fused refill-and-force launch (0 between launches)
  int64_t *dk_copy_ = nullptr;  // the step counter as the two-step launch reads it beside a grid path
  int k2_x0_ = 0, k2_w_ = 1, k2_h_ = 1;
  int64_t k_ = 0;
  bool use_graphs_ = true;
  void *lat_base_ = nullptr;
  hipGraphExec_t gexec_[18] = {};
  std::vector<StepParams> P_host_;
  // checkpoints
  int ckW_ = 0;
  int64_t nck_ = 0;
  size_t ck_lat_bytes_ = 0, ck_grid_bytes_ = 0;
  void *ck_lat_ = nullptr, *ck_grid_ = nullptr;
  bool ck_valid_ = true;
  // adjoint
  bool adj_ready_ = false, adj_done_ = false;
  AdjCtx<T, R> actx_{};
  void *tape_lat_[2] = {nullptr, nullptr};
  R *tape_grid_[2] = {nullptr, nullptr};
  int ntapes_ = 1;
  hipStream_t s_aux_ = nullptr;
  hipEvent_t ev_rec_[2] = {}, ev_rev_[2] = {};
  R *astar_f_ = nullptr, *astar_n_ = nullptr;
  R *alat_[2] = {nullptr, nullptr}, *agrid_[2] = {nullptr, nullptr};
  int adj_lc_ = 0, adj_gc_ = 0;
  R *M2_ = nullptr, *sbf_ = nullptr, *sbn_ = nullptr, *Z1_ = nullptr, *Z2_ = nullptr, *Z3_ = nullptr, *E_ = nullptr;
  R *Vend_ = nullptr;  // outflow ends: adjoints of the two rows at each end
  unsigned char *zf_ = nullptr;
  int *wall_nodes_ = nullptr, *widx_ = nullptr, *acls_ = nullptr;
  unsigned char *ntype_ = nullptr;
  AdjClass<R> *atab_ = nullptr;
  R *wtape_[2] = {nullptr, nullptr};
  int n_wall_ = 0, n_adj_classes_ = 0;
  double *wall_nrm_ = nullptr, *part_ = nullptr, *grad_dev_ = nullptr;
  unsigned long long *counts_scratch_ = nullptr;
  int ex0_ = 0, ey0_ = 0, ew_ = 1, eh_ = 1;
  int slot_refill_ = 0, slot_sub_ = 0, slot_eg_ = 0, slot_sc_ = 0, slot_fg_ = 0, slot_fgg_ = 0,
      nslots_ = 0;
  hipEvent_t tev_adj_[4] = {};
  hipEvent_t tev_adj_ring_[kTimingRing][4] = {};  // lattice adjoint, first sub-step launch
  int aslot_ = 0;
};

#undef ENQ

// Configuration checks shared by all storage types (mirrors the geometric
// requirements stated in hlbm.h).
int validate(const hlbm_config &c, std::string *err, bool ring_ok = false, const double *gx = nullptr,
             const double *gy = nullptr) {
  if (c.nx < 3 || c.ny < 3) { *err = "lattice needs nx, ny >= 3"; return HLBM_E_ARG; }
  if (!(c.tau > 0.5)) { *err = "tau must exceed 1/2"; return HLBM_E_ARG; }
  if (c.bc == HLBM_BC_RING && !ring_ok) {
    *err = "bc HLBM_BC_RING is for the finest level of a multi-level handle";
    return HLBM_E_ARG;
  }
  if (c.bc != HLBM_BC_PERIODIC_X_WALLS_Y && c.bc != HLBM_BC_PERIODIC && c.bc != HLBM_BC_PAPER &&
      c.bc != HLBM_BC_RING) {
    *err = "unknown bc";
    return HLBM_E_ARG;
  }
  if (c.storage < HLBM_FP64 || c.storage > HLBM_FP16_DEV) { *err = "unknown storage"; return HLBM_E_ARG; }
  if (c.max_steps < 0 || c.n_sub < 0 || c.reserved != 0 || c.ckpt_every < 0) { *err = "invalid counts"; return HLBM_E_ARG; }
  if (c.flags & ~HLBM_FLAG_NO_BODY) { *err = "unknown flags"; return HLBM_E_ARG; }
  const bool has_grid = c.nux > 0 || c.nuy > 0;
  if (!has_grid) return HLBM_OK;
  const Derived d = derive(c);
  const double h = c.h_u > 0.0 ? c.h_u : 1.0;
  const bool body = c.b > 0.0 && !(c.flags & HLBM_FLAG_NO_BODY);
  // extents of the grid (uniform spacing h, or the graded columns and rows)
  double hx = (double)(c.nux / 2) * h, hxr = (double)(c.nux - 1 - c.nux / 2) * h;
  double hy = 0.5 * (double)(c.nuy - 1) * h, Tg = h;
  if (gx) {
    if (c.nux < 4 || c.nuy < 4 || (c.nuy % 2)) { *err = "grid needs nux >= 4 and even nuy >= 4"; return HLBM_E_ARG; }
    for (int i = 0; i + 1 < c.nux; ++i)
      if (!(gx[i + 1] > gx[i])) { *err = "graded grid columns must increase"; return HLBM_E_ARG; }
    for (int j = 0; j < c.nuy; ++j)
      if (!(j + 1 == c.nuy || gy[j + 1] > gy[j]) || gy[j] != -gy[c.nuy - 1 - j]) {
        *err = "graded grid rows must increase and be symmetric about the lamina";
        return HLBM_E_ARG;
      }
    hx = -gx[0];
    hxr = gx[c.nux - 1];
    hy = gy[c.nuy - 1];
    Tg = gy[c.nuy / 2] - gy[c.nuy / 2 - 1];
  }
  if (body && std::fabs(c.thickness - Tg) > 1e-12 * Tg) {
    *err = gx ? "lamina thickness must equal the slot rows' spacing" : "lamina thickness must equal h_u";
    return HLBM_E_ARG;
  }
  if (!(1.0 / (double)d.n < 2.0 * d.tau_u)) { *err = "grid sub-step violates Delta t_u < 2 tau_u"; return HLBM_E_ARG; }
  if (c.nux < 4 || c.nuy < 4 || (c.nuy % 2)) { *err = "grid needs nux >= 4 and even nuy >= 4"; return HLBM_E_ARG; }
  if (d.xc - hx < 1.0 || d.xc + hxr > (double)c.nx - 2.0) { *err = "grid leaves the lattice in x"; return HLBM_E_ARG; }
  if (c.bc != HLBM_BC_PERIODIC &&
      (d.yc - hy - std::fabs(d.A) < 1.0 || d.yc + hy + std::fabs(d.A) > (double)c.ny - 2.0)) {
    *err = "grid motion leaves the lattice in y";
    return HLBM_E_ARG;
  }
  if (body && (0.5 * c.b + 1.0 > hx - kMargin - 1.0 || 0.5 * c.b + 1.0 > hxr - kMargin - 1.0 ||
               0.5 * Tg + 1.0 > hy - kMargin - 1.0)) {
    *err = "lamina does not fit inside the fictitious rectangle";
    return HLBM_E_ARG;
  }
  if (!(std::fabs(d.A * d.omega) < 1.0)) { *err = "lamina speed must stay below one lattice unit per step"; return HLBM_E_ARG; }
  return HLBM_OK;
}


// Many cases advanced together. Every phase of the structured step is one
// launch over the work list of all running cases (case-batched kernels pick
// each case's buffers from its step counter), and steps_per_graph steps are
// captured as one HIP graph. Cases stop at their own max_steps; a case whose
// force becomes non-finite stops at once (the kernels skip it) and is retired
// at the next host check. Lists and graphs are rebuilt when the set of
// running cases changes.
template <class T, class R>
class Batch final : public CaseBase {
 public:
  ~Batch() override { release(); }

  int init(const hlbm_config *cfgs, int n) {
    for (int i = 0; i < n; ++i) {
      auto c = std::make_unique<Case<T, R>>();
      const int rc = c->init(cfgs[i], false);
      if (rc != HLBM_OK) {
        err = "case " + std::to_string(i) + ": " + c->err;
        return rc;
      }
      cases_.push_back(std::move(c));
    }
    HIPCHK(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
    HIPCHK(hipEventCreate(&ev0_));
    HIPCHK(hipEventCreate(&ev1_));
    std::vector<CaseView<T, R>> v(n);
    for (int i = 0; i < n; ++i) v[i] = cases_[i]->batched_view();
    HIPCHK(hipMalloc(&views_, n * sizeof(CaseView<T, R>)));
    HIPCHK(hipMemcpy(views_, v.data(), n * sizeof(CaseView<T, R>), hipMemcpyHostToDevice));
    tuning_ = {8, kLatticeThreads, kLatticeRows, -1, 1, -1, 0, 0, 0.0};
    tail_n_ = std::max(1, n / 8);
    return HLBM_OK;
  }

  CaseBase *sub(int id) override {
    return id >= 0 && id < (int)cases_.size() ? cases_[id].get() : nullptr;
  }

  int step(int64_t nsteps) override {
    if (nsteps < 0) return fail(HLBM_E_ARG, "nsteps < 0");
    int64_t done = 0;
    while (done < nsteps) {
      std::vector<int> act;
      int64_t room = nsteps - done;
      for (int i = 0; i < (int)cases_.size(); ++i) {
        if (retired_.count(i)) continue;
        const int64_t left = cases_[i]->max_steps() - cases_[i]->steps_taken();
        if (left <= 0) continue;
        act.push_back(i);
        room = std::min(room, left);
      }
      if (act.empty()) break;
      int rc = run(act, room);
      if (rc != HLBM_OK) return rc;
      done += room;
    }
    return HLBM_OK;
  }

  int tune(int trial_steps, hlbm_tuning *t) override {
    if (!t || trial_steps < 0) return fail(HLBM_E_ARG, "invalid tuning request");
    for (auto &c : cases_)
      if (c->steps_taken() != 0) return fail(HLBM_E_STATE, "tuning must precede the first step");
    if (trial_steps == 0) {
      if (t->steps_per_graph < 1 || t->steps_per_graph > 64 || !valid_lattice_shape(*t) ||
          t->substep_variant < -1 || t->substep_variant >= kSubstepVariants || t->order < 0 || t->order > 1 ||
          t->tail_variant < -1 || t->tail_variant >= kSubstepVariants || t->persistent < 0 || t->persistent > 2 ||
          t->persistent_groups < 0)
        return fail(HLBM_E_ARG, "invalid schedule");
      tuning_ = *t;
      tuning_.ms_per_step = 0.0;
      invalidate();
      *t = tuning_;
      return HLBM_OK;
    }
    // snapshot of every case's state at step 0
    std::vector<void *> snap;
    for (auto &c : cases_) {
      void *lat[2], *grid[2];
      size_t lb, gb;
      c->buffers(lat, grid, &lb, &gb);
      void *p = nullptr;
      HIPCHK(hipMalloc(&p, lb + gb));
      snap.push_back(p);
      HIPCHK(hipMemcpy(p, lat[0], lb, hipMemcpyDeviceToDevice));
      HIPCHK(hipMemcpy((char *)p + lb, grid[0], gb, hipMemcpyDeviceToDevice));
    }
    std::vector<int> all;
    for (int i = 0; i < (int)cases_.size(); ++i)
      if (cases_[i]->max_steps() >= trial_steps) all.push_back(i);
    // one choice at a time, the others held at the best found so far
    hlbm_tuning best = tuning_;
    double best_ms = 1e300;
    int rc = HLBM_OK;
    auto trial = [&](hlbm_tuning cand) {
      if (rc != HLBM_OK) return;
      tuning_ = cand;
      invalidate();
      float ms = 0.f;
      rc = timed_trial(all, trial_steps, &ms);
      if (rc == HLBM_OK) rc = restore(snap);
      if (rc == HLBM_OK && ms / trial_steps < best_ms) {
        best_ms = ms / trial_steps;
        best = cand;
      }
    };
    auto cand = [](hlbm_tuning b) {
      b.tail_variant = -1;
      b.ms_per_step = 0.0;
      return b;
    };
    for (int g : {4, 8, 16}) {
      hlbm_tuning c = cand(best);
      c.steps_per_graph = g;
      trial(c);
    }
    const hlbm_tuning after_g = best;
    for (int lt : {128, 256})
      for (int rows : {1, 2, 4})
        if (lt != after_g.lattice_threads || rows != after_g.lattice_rows) {
          hlbm_tuning c = cand(after_g);
          c.lattice_threads = lt;
          c.lattice_rows = rows;
          trial(c);
        }
    const hlbm_tuning after_l = best;
    for (int sv = 0; sv < kSubstepVariants; ++sv)
      if (sv != (after_l.substep_variant < 0 ? default_substep_variant<R>() : after_l.substep_variant)) {
        hlbm_tuning c = cand(after_l);
        c.substep_variant = sv;
        trial(c);
      }
    const hlbm_tuning after_s = best;
    {
      hlbm_tuning c = cand(after_s);
      c.order = 1 - after_s.order;
      trial(c);
    }
    // one persistent cooperative launch per run instead of the graphs, in
    // each of its sub-step variants, then its workgroup count
    const hlbm_tuning after_o = best;
    for (int sv = kPersistentFirst; sv <= kPersistentLast; ++sv) {
      hlbm_tuning c = cand(after_o);
      c.persistent = 1;
      c.persistent_groups = 0;
      c.substep_variant = sv;
      trial(c);
    }
    if (best.persistent == 1) {
      const hlbm_tuning after_p = best;
      for (int g : {256, 512, 1024}) {
        hlbm_tuning c = cand(after_p);
        c.persistent_groups = g;
        trial(c);
      }
    }
    const double all_ms = best_ms;
    // the last few cases (the longest runs) often want another sub-step
    // kernel than the full set, or the persistent launch: time them alone
    std::vector<int> tail(all);
    std::sort(tail.begin(), tail.end(),
              [&](int a, int b) { return cases_[a]->max_steps() > cases_[b]->max_steps(); });
    if ((int)tail.size() > tail_n_) tail.resize(tail_n_);
    int tail_sv = -1, tail_persistent = 0;
    if (rc == HLBM_OK && !tail.empty() && tail.size() < all.size()) {
      float tail_best = 3e38f;
      for (int mode = best.persistent == 1 ? 1 : 0; mode <= 1 && rc == HLBM_OK; ++mode)
        for (int sv = mode ? kPersistentFirst : 0; sv <= (mode ? kPersistentLast : kSubstepVariants - 1) &&
                                                    rc == HLBM_OK;
             ++sv) {
          tuning_ = best;
          tuning_.persistent = mode;
          tuning_.substep_variant = sv;
          invalidate();
          float ms = 0.f;
          rc = timed_trial(tail, trial_steps, &ms);
          if (rc == HLBM_OK) rc = restore(snap);
          if (rc == HLBM_OK && ms < tail_best) {
            tail_best = ms;
            tail_sv = sv;
            tail_persistent = mode;
          }
        }
    }
    for (void *p : snap) (void)hipFree(p);
    if (rc != HLBM_OK) return rc;
    tuning_ = best;
    tuning_.tail_variant = tail_sv;
    if (best.persistent == 0 && tail_persistent) tuning_.persistent = 2;
    tuning_.ms_per_step = all_ms;
    invalidate();
    *t = tuning_;
    return HLBM_OK;
  }

  int get_state(int, void *, size_t) override { return fail(HLBM_E_ARG, "select a case"); }
  int set_state(int, const void *, size_t) override { return fail(HLBM_E_ARG, "select a case"); }
  int force(double *, int64_t, int64_t *, double, double, double *) override {
    return fail(HLBM_E_ARG, "select a case");
  }
  int info(hlbm_info *) override { return fail(HLBM_E_ARG, "select a case"); }
  int stencil(int, int32_t *, double *, double *) override {
    return fail(HLBM_E_UNSUPPORTED, "stencils are per case: create the case alone");
  }
  int timing(int) override { return fail(HLBM_E_UNSUPPORTED, "per-kernel timing is per single case"); }
  int timing_get(int, double *, int64_t *) override {
    return fail(HLBM_E_UNSUPPORTED, "per-kernel timing is per single case");
  }
  int adjoint(const double *, int64_t, double *) override {
    return fail(HLBM_E_UNSUPPORTED, "the adjoint runs on single cases");
  }

 private:
  struct List {
    int4 *d = nullptr;
    int n = 0;
  };

  int fail(int code, const std::string &msg) {
    err = msg;
    return code;
  }

  void invalidate() {
    if (gexec_) (void)hipGraphExecDestroy(gexec_);
    gexec_ = nullptr;
    listed_.clear();
    if (pitems_) (void)hipFree(pitems_);
    if (pprog_) (void)hipFree(pprog_);
    pitems_ = nullptr;
    pprog_ = nullptr;
    plisted_.clear();
  }

  void release() {
    if (s_) (void)hipStreamSynchronize(s_);
    invalidate();
    for (auto &l : lists_)
      if (l.d) (void)hipFree(l.d);
    lists_.clear();
    if (views_) (void)hipFree(views_);
    if (ev0_) (void)hipEventDestroy(ev0_);
    if (ev1_) (void)hipEventDestroy(ev1_);
    if (s_) (void)hipStreamDestroy(s_);
    cases_.clear();
  }

  // reorders a work list so that XCD x (workgroup b runs on XCD b % 8) gets
  // a contiguous chunk of it
  static void deal_to_xcds(std::vector<int4> &v) {
    const size_t n = v.size(), per = (n + 7) / 8;
    std::vector<int4> out;
    out.reserve(n);
    for (size_t b = 0; b < 8 * per; ++b) {
      const size_t src = (b % 8) * per + b / 8;
      if (src < n) out.push_back(v[src]);
    }
    v.swap(out);
  }

  hipError_t upload_list(std::vector<int4> &v, List &l) {
    if (tuning_.order == 1) deal_to_xcds(v);
    l.n = (int)v.size();
    if (l.d) (void)hipFree(l.d);
    l.d = nullptr;
    if (v.empty()) return hipSuccess;
    hipError_t e = hipMalloc(&l.d, v.size() * sizeof(int4));
    if (e == hipSuccess) e = hipMemcpy(l.d, v.data(), v.size() * sizeof(int4), hipMemcpyHostToDevice);
    return e;
  }

  bool is_tail(const std::vector<int> &act) const { return (int)act.size() <= tail_n_; }

  // the sub-step kernel for this set of running cases
  int variant_for(const std::vector<int> &act) const {
    const int sv = (tuning_.tail_variant >= 0 && is_tail(act)) ? tuning_.tail_variant : tuning_.substep_variant;
    return sv < 0 ? default_substep_variant<R>() : sv;
  }

  bool persistent_for(const std::vector<int> &act) const {
    return tuning_.persistent == 1 || (tuning_.persistent == 2 && is_tail(act));
  }

  // work items and phases of one persistent step over the running cases:
  // the items of every phase built for workgroups of the persistent
  // kernel's width (one lattice row per stream-collide item), in the order
  // of the graph path's launches
  hipError_t build_persistent(const std::vector<int> &act) {
    const int sv = variant_for(act);
    pv_ = (sv >= kPersistentFirst && sv <= kPersistentLast) ? sv : kPersistentDefault;
    const int nt = Kernels<T, R>::persistent_threads(pv_);
    std::vector<int4> items;
    std::vector<BatchPhase> prog;
    int widest = 1;
    auto phase = [&](BatchKernel which, int m0, auto &&fill) {
      const int first = (int)items.size();
      for (int c : act) fill(c, cases_[c]->batched_view());
      const int n = (int)items.size() - first;
      if (n > 0) prog.push_back(BatchPhase{(int)which, first, n, m0});
      widest = std::max(widest, n);
    };
    phase(BatchKernel::LatticeFromGrid, 0, [&](int c, const CaseView<T, R> &v) {
      for (int by = 0; by < v.k2_h; ++by)
        for (int bx = 0; bx < (v.k2_w + nt - 1) / nt; ++bx) items.push_back(make_int4(c, bx, by, 0));
    });
    phase(BatchKernel::StreamCollide, 0, [&](int c, const CaseView<T, R> &v) {
      for (int by = 0; by < v.ny; ++by)
        for (int bx = 0; bx < (v.nx + nt - 1) / nt; ++bx) items.push_back(make_int4(c, bx, by, 0));
    });
    phase(BatchKernel::InterfaceDonors, 0, [&](int c, const CaseView<T, R> &v) {
      for (int bx = 0; bx < (4 * v.n_iface + nt - 1) / nt; ++bx) items.push_back(make_int4(c, bx, 0, 0));
    });
    int lmax = 0;
    for (int c : act) {
      const CaseView<T, R> v = cases_[c]->batched_view();
      lmax = std::max(lmax, (v.n_sub + kSubstepBlock - 1) / kSubstepBlock);
    }
    int tx, ty;
    substep_tile(pv_, &tx, &ty);
    for (int i = 0; i < lmax; ++i)
      phase(BatchKernel::GridSubsteps, i * kSubstepBlock, [&](int c, const CaseView<T, R> &v) {
        if ((v.n_sub + kSubstepBlock - 1) / kSubstepBlock <= i) return;
        const int tiles = ((v.nux + tx - 1) / tx) * ((v.nuy + ty - 1) / ty);
        for (int t = 0; t < tiles; ++t) items.push_back(make_int4(c, t, 0, 0));
      });
    phase(BatchKernel::Refill, 0, [&](int c, const CaseView<T, R> &v) {
      for (int bx = 0; bx < (v.nnode + nt - 1) / nt; ++bx) items.push_back(make_int4(c, bx, 0, 0));
    });
    phase(BatchKernel::Force, 0, [&](int c, const CaseView<T, R> &) { items.push_back(make_int4(c, 0, 0, 0)); });
    hipError_t e = hipMalloc(&pitems_, items.size() * sizeof(int4));
    if (e == hipSuccess) e = hipMemcpy(pitems_, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&pprog_, prog.size() * sizeof(BatchPhase));
    if (e == hipSuccess)
      e = hipMemcpy(pprog_, prog.data(), prog.size() * sizeof(BatchPhase), hipMemcpyHostToDevice);
    pnphase_ = (int)prog.size();
    // more workgroups than the widest phase has items would only wait
    pgroups_ = tuning_.persistent_groups > 0 ? std::min(tuning_.persistent_groups, widest) : widest;
    plisted_ = act;
    return e;
  }

  hipError_t ensure_persistent(const std::vector<int> &act) {
    if (pitems_ && act == plisted_) return hipSuccess;
    invalidate();
    return build_persistent(act);
  }

  // m steps of the running cases in cooperative launches of at most
  // kPersistentChunk steps each
  hipError_t launch_persistent(int64_t m) {
    for (int64_t s = 0; s < m; s += kPersistentChunk) {
      const int n = (int)std::min<int64_t>(kPersistentChunk, m - s);
      hipError_t e = Kernels<T, R>::batched_persistent(views_, pitems_, pprog_, pnphase_, n, pv_, pgroups_, s_);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }

  // work lists of the running cases: stream-collide, lattice-from-grid,
  // donors, refill, force, then one per sub-step launch
  hipError_t build_lists(const std::vector<int> &act) {
    sv_ = variant_for(act);
    for (auto &l : lists_)
      if (l.d) (void)hipFree(l.d);
    lists_.assign(5, List{});
    int lmax = 0;
    std::vector<int4> k1, k2, dn, rf, fo;
    const int lt = tuning_.lattice_threads, rows = tuning_.lattice_rows;
    for (int c : act) {
      const CaseView<T, R> v = cases_[c]->batched_view();
      for (int by = 0; by < (v.ny + rows - 1) / rows; ++by)
        for (int bx = 0; bx < (v.nx + lt - 1) / lt; ++bx) k1.push_back(make_int4(c, bx, by, 0));
      for (int by = 0; by < v.k2_h; ++by)
        for (int bx = 0; bx < (v.k2_w + 255) / 256; ++bx) k2.push_back(make_int4(c, bx, by, 0));
      for (int bx = 0; bx < (4 * v.n_iface + 255) / 256; ++bx) dn.push_back(make_int4(c, bx, 0, 0));
      for (int bx = 0; bx < (v.nnode + 255) / 256; ++bx) rf.push_back(make_int4(c, bx, 0, 0));
      fo.push_back(make_int4(c, 0, 0, 0));
      lmax = std::max(lmax, (v.n_sub + kSubstepBlock - 1) / kSubstepBlock);
    }
    hipError_t e = upload_list(k1, lists_[0]);
    if (e == hipSuccess) e = upload_list(k2, lists_[1]);
    if (e == hipSuccess) e = upload_list(dn, lists_[2]);
    if (e == hipSuccess) e = upload_list(rf, lists_[3]);
    if (e == hipSuccess) e = upload_list(fo, lists_[4]);
    for (int i = 0; i < lmax && e == hipSuccess; ++i) {
      std::vector<int4> sl;
      for (int c : act) {
        const CaseView<T, R> v = cases_[c]->batched_view();
        if ((v.n_sub + kSubstepBlock - 1) / kSubstepBlock <= i) continue;
        int tx, ty;
        substep_tile(sv_, &tx, &ty);
        const int tiles = ((v.nux + tx - 1) / tx) * ((v.nuy + ty - 1) / ty);
        for (int t = 0; t < tiles; ++t) sl.push_back(make_int4(c, t, 0, 0));
      }
      lists_.push_back(List{});
      e = upload_list(sl, lists_.back());
    }
    listed_ = act;
    return e;
  }

  void enqueue_step() {
    using K = Kernels<T, R>;
    K::batched(BatchKernel::LatticeFromGrid, views_, lists_[1].d, lists_[1].n, 0, 256, s_);
    K::batched(BatchKernel::StreamCollide, views_, lists_[0].d, lists_[0].n, 0, tuning_.lattice_threads, s_,
               tuning_.lattice_rows);
    K::batched(BatchKernel::InterfaceDonors, views_, lists_[2].d, lists_[2].n, 0, 256, s_);
    for (size_t i = 5; i < lists_.size(); ++i)
      K::batched(BatchKernel::GridSubsteps, views_, lists_[i].d, lists_[i].n, (int)(i - 5) * kSubstepBlock, sv_,
                 s_);
    K::batched(BatchKernel::Refill, views_, lists_[3].d, lists_[3].n, 0, 256, s_);
    K::batched(BatchKernel::Force, views_, lists_[4].d, lists_[4].n, 0, 256, s_);
  }

  hipError_t ensure_graph(const std::vector<int> &act) {
    if (gexec_ && act == listed_) return hipSuccess;
    invalidate();
    hipError_t e = build_lists(act);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    for (int i = 0; i < tuning_.steps_per_graph; ++i) enqueue_step();
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s_, &g);
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&gexec_, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
  }

  // m steps of the running cases act (none of them ends before m steps)
  int run(const std::vector<int> &act, int64_t m) {
    if (persistent_for(act)) {
      HIPCHK(ensure_persistent(act));
      HIPCHK(launch_persistent(m));
    } else {
      HIPCHK(ensure_graph(act));
      int64_t s = 0;
      for (; s + tuning_.steps_per_graph <= m; s += tuning_.steps_per_graph) HIPCHK(hipGraphLaunch(gexec_, s_));
      for (; s < m; ++s) enqueue_step();
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s_));
    for (int c : act) {
      int64_t k = 0;
      HIPCHK(hipMemcpy(&k, cases_[c]->step_counter(), sizeof(k), hipMemcpyDeviceToHost));
      const int64_t adv = k - cases_[c]->steps_taken();
      cases_[c]->advance_host(adv);
      if (adv != m) retired_.insert(c);  // stopped early: non-finite force
    }
    return HLBM_OK;
  }

  int timed_trial(const std::vector<int> &act, int steps, float *ms) {
    if (persistent_for(act)) {
      HIPCHK(ensure_persistent(act));
      HIPCHK(launch_persistent(tuning_.steps_per_graph));  // untimed
      HIPCHK(hipEventRecord(ev0_, s_));
      HIPCHK(launch_persistent(steps));
    } else {
      HIPCHK(ensure_graph(act));
      // one untimed graph launch, then the timed steps
      HIPCHK(hipGraphLaunch(gexec_, s_));
      HIPCHK(hipEventRecord(ev0_, s_));
      int s = 0;
      for (; s + tuning_.steps_per_graph <= steps; s += tuning_.steps_per_graph) HIPCHK(hipGraphLaunch(gexec_, s_));
      for (; s < steps; ++s) enqueue_step();
    }
    HIPCHK(hipEventRecord(ev1_, s_));
    HIPCHK(hipEventSynchronize(ev1_));
    HIPCHK(hipEventElapsedTime(ms, ev0_, ev1_));
    return HLBM_OK;
  }

  // back to the snapshot taken at step 0
  int restore(const std::vector<void *> &snap) {
    HIPCHK(hipStreamSynchronize(s_));
    for (size_t i = 0; i < cases_.size(); ++i) {
      void *lat[2], *grid[2];
      size_t lb, gb;
      cases_[i]->buffers(lat, grid, &lb, &gb);
      HIPCHK(hipMemcpy(lat[0], snap[i], lb, hipMemcpyDeviceToDevice));
      HIPCHK(hipMemcpy(grid[0], (char *)snap[i] + lb, gb, hipMemcpyDeviceToDevice));
      HIPCHK(hipMemset(cases_[i]->step_counter(), 0, sizeof(int64_t)));
      HIPCHK(hipMemset(cases_[i]->flag(), 0, sizeof(int)));
      HIPCHK(hipMemset(cases_[i]->refill_counters(), 0, 2 * sizeof(unsigned long long)));
    }
    return HLBM_OK;
  }

  std::vector<std::unique_ptr<Case<T, R>>> cases_;
  std::set<int> retired_;
  CaseView<T, R> *views_ = nullptr;
  std::vector<List> lists_;
  std::vector<int> listed_;
  hipGraphExec_t gexec_ = nullptr;
  hipStream_t s_ = nullptr;
  hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
  hlbm_tuning tuning_{};
  int tail_n_ = 1;  // at most this many running cases: the tail's sub-step variant
  int sv_ = 0;      // sub-step variant of the current work lists
  // persistent launch: items and phases of the running cases plisted_
  int4 *pitems_ = nullptr;
  BatchPhase *pprog_ = nullptr;
  std::vector<int> plisted_;
  int pnphase_ = 0, pgroups_ = 1, pv_ = kPersistentDefault;
  static constexpr int kPersistentFirst = 4, kPersistentLast = 7, kPersistentDefault = 5;
  static constexpr int64_t kPersistentChunk = 256;
};

// Nested structured refinement levels. Levels 0 .. L-2 are plain lattices
// owned here; the finest is a Case (lattice with or without the body-fitted
// grid) whose outermost ring of nodes is written from level L-2. One step
// advances level 0 by one step and level l by 2^l steps, recursively: level
// l streams and collides (skipping the nodes the finer level covers),
// records the pre-collision moments on the perimeter of the finer level's
// box, runs two steps of the finer level with its ring interpolated at
// t and t + 1/2, and takes its nodes one inside the box from the finer
// level at t + 1. Everything runs on the finest case's stream; one step of
// level 0 is captured as one HIP graph per buffer arrangement of level 0
// (every finer level takes an even number of steps, so its buffers are back
// in place).
template <class T, class R>
class MultiLevel final : public CaseBase {
 public:
  ~MultiLevel() override { release(); }

  int init(const hlbm_config &fine, const hlbm_levels &lv) {
    L_ = lv.nlevels;
    fine_cfg_ = fine;
    fine_ = std::make_unique<Case<T, R>>();
    int rc = fine_->init(fine);
    if (rc != HLBM_OK) {
      err = fine_->err;
      return rc;
    }
    s_ = fine_->stream();
    // equal viscosity: tau - 1/2 halves from each level to the next coarser
    std::vector<double> taus(L_);
    taus[L_ - 1] = fine.tau;
    for (int l = L_ - 2; l >= 0; --l) taus[l] = 0.5 + 0.5 * (taus[l + 1] - 0.5);
    int nx = lv.nx0, ny = lv.ny0;
    for (int l = 0; l < L_ - 1; ++l) {
      Level &c = lev_[l];
      c.nx = nx;
      c.ny = ny;
      c.bc = l == 0 ? lv.bc0 : 3;
      c.tau = taus[l];
      c.box = {lv.box[l][0], lv.box[l][1], lv.box[l][2], lv.box[l][3]};
      c.plane = lattice_plane(nx, ny);
      for (int i = 0; i < 2; ++i) {
        HIPCHK(alloc(&c.lat[i], 9 * c.plane * sizeof(T)));
        HIPCHK(alloc(&c.m[i], 12 * (size_t)c.box.perimeter() * sizeof(R)));
        Kernels<T, R>::fill_rest((T *)c.lat[i], c.plane, nullptr, 0, s_);
      }
      c.base = c.lat[0];
      LevelKernels<T, R>::box_moments((const T *)c.lat[0], c.nx, c.ny, c.plane, c.bc, c.box, (R *)c.m[0], s_);
      nx = 2 * c.box.W() + 1;
      ny = 2 * c.box.H() + 1;
    }
    use_graphs_ = std::getenv("HLBM_NO_GRAPHS") == nullptr;
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s_));
    return HLBM_OK;
  }

  int step(int64_t nsteps) override {
    if (nsteps < 0) return fail(HLBM_E_ARG, "nsteps < 0");
    const int64_t per = (int64_t)1 << (L_ - 1);
    if (fine_->has_grid() && fine_->steps_taken() + nsteps * per > fine_->max_steps())
      return fail(HLBM_E_ARG, "force history of the finest level would exceed max_steps");
    for (int64_t i = 0; i < nsteps; ++i) {
      if (use_graphs_) {
        hipGraphExec_t g = nullptr;
        HIPCHK(graph(&g));
        HIPCHK(hipGraphLaunch(g, s_));
        // level 0 took one step, every finer level an even number
        std::swap(lev_[0].lat[0], lev_[0].lat[1]);
        std::swap(lev_[0].m[0], lev_[0].m[1]);
        fine_->advance_host(per);
      } else {
        HIPCHK(advance(0));
      }
    }
    HIPCHK(hipStreamSynchronize(s_));
    int flag = 0;
    HIPCHK(hipMemcpy(&flag, fine_->flag(), sizeof(int), hipMemcpyDeviceToHost));
    if (flag & 2) return fail(HLBM_E_UNSTABLE, "a density of the finest level became non-positive or not a number");
    if (flag) return fail(HLBM_E_UNSTABLE, "non-finite force on the lamina");
    return HLBM_OK;
  }

  int get_state(int which, void *buf, size_t bytes) override {
    const int l = which == HLBM_STATE_LATTICE ? L_ - 1 : which - HLBM_STATE_LEVEL;
    if (which != HLBM_STATE_LATTICE && (l < 0 || l >= L_)) {
      if (which == HLBM_STATE_GRID) return relay(fine_->get_state(which, buf, bytes));
      return fail(HLBM_E_ARG, "unknown state selector");
    }
    if (l == L_ - 1) return relay(fine_->get_state(HLBM_STATE_LATTICE, buf, bytes));
    const Level &c = lev_[l];
    const size_t nodes = (size_t)c.nx * c.ny;
    if (bytes != 9 * nodes * sizeof(double)) return fail(HLBM_E_ARG, "level state size mismatch");
    HIPCHK(hipStreamSynchronize(s_));
    double *tmp = nullptr;
    HIPCHK(hipMalloc(&tmp, bytes));
    Kernels<T, R>::lattice_to_f64((const T *)c.lat[0], tmp, c.plane, nodes, s_);
    hipError_t e = hipMemcpyAsync(buf, tmp, bytes, hipMemcpyDeviceToHost, s_);
    if (e == hipSuccess) e = hipStreamSynchronize(s_);
    (void)hipFree(tmp);
    HIPCHK(e);
    return HLBM_OK;
  }

  int get_state_noalloc(int which, void *buf, size_t bytes) override {
    if (which != HLBM_STATE_LATTICE && which != HLBM_STATE_GRID)
      return fail(HLBM_E_ARG, "only the finest lattice and the grid are read without allocating");
    return relay(fine_->get_state_noalloc(which, buf, bytes));
  }

  // A level is set as a steady state: both of its buffers, and the moments
  // on the perimeter of the finer level's box as those of the current time.
  int set_state(int which, const void *buf, size_t bytes) override {
    const int l = which == HLBM_STATE_LATTICE ? L_ - 1 : which - HLBM_STATE_LEVEL;
    if (which != HLBM_STATE_LATTICE && (l < 0 || l >= L_)) {
      if (which == HLBM_STATE_GRID) return relay(fine_->set_state(which, buf, bytes));
      return fail(HLBM_E_ARG, "state cannot be set");
    }
    if (l == L_ - 1) {
      const int rc = fine_->set_state(HLBM_STATE_LATTICE, buf, bytes);
      if (rc != HLBM_OK) return relay(rc);
      HIPCHK(hipMemcpy(fine_->lattice_buffer(1), fine_->lattice_buffer(0), 9 * fine_->plane() * sizeof(T),
                       hipMemcpyDeviceToDevice));
      return HLBM_OK;
    }
    Level &c = lev_[l];
    const size_t nodes = (size_t)c.nx * c.ny;
    if (bytes != 9 * nodes * sizeof(double)) return fail(HLBM_E_ARG, "level state size mismatch");
    HIPCHK(hipStreamSynchronize(s_));
    double *tmp = nullptr;
    HIPCHK(hipMalloc(&tmp, bytes));
    hipError_t e = hipMemcpyAsync(tmp, buf, bytes, hipMemcpyHostToDevice, s_);
    if (e == hipSuccess) {
      for (int i = 0; i < 2; ++i) Kernels<T, R>::lattice_from_f64(tmp, (T *)c.lat[i], c.plane, nodes, s_);
      LevelKernels<T, R>::box_moments((const T *)c.lat[0], c.nx, c.ny, c.plane, c.bc, c.box, (R *)c.m[0], s_);
      e = hipGetLastError();
      if (e == hipSuccess) e = hipStreamSynchronize(s_);
    }
    (void)hipFree(tmp);
    HIPCHK(e);
    return HLBM_OK;
  }

  int force(double *hist, int64_t cap, int64_t *n_out, double t0, double t1, double th[2]) override {
    return relay(fine_->force(hist, cap, n_out, t0, t1, th));
  }
  int info(hlbm_info *o) override { return relay(fine_->info(o)); }
  int stencil(int kmax, int32_t *nbr, double *S, double *C) override {
    return relay(fine_->stencil(kmax, nbr, S, C));
  }
  int timing(int) override { return fail(HLBM_E_UNSUPPORTED, "per-kernel timing of a multi-level handle"); }
  int timing_get(int, double *, int64_t *) override {
    return fail(HLBM_E_UNSUPPORTED, "per-kernel timing of a multi-level handle");
  }
  int adjoint(const double *, int64_t, double *) override {
    return fail(HLBM_E_UNSUPPORTED, "adjoint of a multi-level handle");
  }

  // the finest case's autotuner; its stream-collide shape serves every level
  int tune(int trial_steps, hlbm_tuning *t) override {
    HIPCHK(hipStreamSynchronize(s_));
    const int rc = fine_->tune(trial_steps, t);
    if (rc != HLBM_OK) return relay(rc);
    threads_ = t->lattice_threads;
    rows_ = t->lattice_rows;
    order_ = t->order;
    drop_graphs();
    return HLBM_OK;
  }

  int shape(int l, int *nx, int *ny, double *tau) const {
    if (l < 0 || l >= L_) return HLBM_E_ARG;
    if (l == L_ - 1) {
      *nx = fine_cfg_.nx;
      *ny = fine_cfg_.ny;
      *tau = fine_cfg_.tau;
    } else {
      *nx = lev_[l].nx;
      *ny = lev_[l].ny;
      *tau = lev_[l].tau;
    }
    return HLBM_OK;
  }

 private:
  struct Level {
    int nx = 0, ny = 0, bc = 0;
    double tau = 0.0;
    size_t plane = 0;
    LevelBox box{};
    void *lat[2] = {nullptr, nullptr};  // post-collision state at t (0) and t - 1 (1)
    void *m[2] = {nullptr, nullptr};    // perimeter moments at t (0) and t + 1 (1)
    void *base = nullptr;
  };

  CaseView<T, R> level_view(int l) const {
    const Level &c = lev_[l];
    CaseView<T, R> v{};
    v.A = (const T *)c.lat[0];
    v.B = (T *)c.lat[1];
    v.nx = c.nx;
    v.ny = c.ny;
    v.plane = c.plane;
    v.bc = c.bc;
    v.inv_tau = (R)(1.0 / c.tau);
    v.wx0 = 0;
    v.wy0 = 0;
    v.ww = c.nx;
    v.wh = c.ny;
    v.sx0 = c.box.x0;
    v.sx1 = c.box.x1;
    v.sy0 = c.box.y0;
    v.sy1 = c.box.y1;
    return v;
  }

  void child(int l, void **cur, void **prev, int *nx, int *ny, size_t *plane, double *tau) const {
    if (l == L_ - 1) {
      *cur = fine_->lattice_buffer(0);
      *prev = fine_->lattice_buffer(1);
      *nx = fine_cfg_.nx;
      *ny = fine_cfg_.ny;
      *plane = fine_->plane();
      *tau = fine_cfg_.tau;
    } else {
      const Level &c = lev_[l];
      *cur = c.lat[0];
      *prev = c.lat[1];
      *nx = c.nx;
      *ny = c.ny;
      *plane = c.plane;
      *tau = c.tau;
    }
  }

  // enqueue one step of level l (and 2^(l'-l) of every finer level l')
  hipError_t advance(int l) {
    if (l == L_ - 1) return fine_->enqueue_one();
    Level &c = lev_[l];
    Kernels<T, R>::stream_collide(level_view(l), s_, nullptr, nullptr, threads_, rows_, order_);
    std::swap(c.lat[0], c.lat[1]);
    LevelKernels<T, R>::box_moments((const T *)c.lat[1], c.nx, c.ny, c.plane, c.bc, c.box, (R *)c.m[1], s_);
    void *fc, *fp;
    int nxf, nyf;
    size_t planef;
    double tauf;
    child(l + 1, &fc, &fp, &nxf, &nyf, &planef, &tauf);
    // f^neq scales with tau Delta x between the levels
    const double kf = (1.0 - 1.0 / tauf) * (tauf / (2.0 * c.tau));
    const double kc = (1.0 - 1.0 / c.tau) * (2.0 * c.tau / tauf);
    for (int h = 0; h < 2; ++h) {
      child(l + 1, &fc, &fp, &nxf, &nyf, &planef, &tauf);
      LevelKernels<T, R>::prolong((const R *)c.m[0], (const R *)c.m[1], c.box, 0.5 * (double)h, kf, (T *)fc, nxf, nyf,
                                  planef, s_);
      const hipError_t e = advance(l + 1);
      if (e != hipSuccess) return e;
    }
    child(l + 1, &fc, &fp, &nxf, &nyf, &planef, &tauf);
    LevelKernels<T, R>::restrict_level((const T *)fp, nxf, nyf, planef, c.box, kc, (T *)c.lat[0], c.nx, c.plane,
                                       s_);
    std::swap(c.m[0], c.m[1]);
    return hipGetLastError();
  }

  hipError_t graph(hipGraphExec_t *out) {
    const int key = lev_[0].lat[0] == lev_[0].base ? 0 : 1;
    if (gexec_[key]) {
      *out = gexec_[key];
      return hipSuccess;
    }
    Level saved[kMaxLevels];
    for (int l = 0; l < L_ - 1; ++l) saved[l] = lev_[l];
    const auto fl = fine_->layout();
    hipError_t e = hipStreamBeginCapture(s_, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t e2 = advance(0);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s_, &g);
    for (int l = 0; l < L_ - 1; ++l) lev_[l] = saved[l];
    fine_->set_layout(fl);
    if (e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return e2;
    }
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&gexec_[key], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
    *out = gexec_[key];
    return hipSuccess;
  }

  void drop_graphs() {
    for (auto &g : gexec_) {
      if (g) (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  }

  template <class P>
  hipError_t alloc(P **p, size_t bytes) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) owned_.push_back(q);
    *p = (P *)q;
    return e;
  }

  void release() {
    if (s_) (void)hipStreamSynchronize(s_);
    drop_graphs();
    for (void *p : owned_) (void)hipFree(p);
    owned_.clear();
  }

  int fail(int code, const char *msg) {
    err = msg;
    return code;
  }
  int relay(int rc) {
    if (rc != HLBM_OK) err = fine_->err;
    return rc;
  }

  static constexpr int kMaxLevels = HLBM_MAX_LEVELS;
  int L_ = 0;
  hlbm_config fine_cfg_{};
  std::unique_ptr<Case<T, R>> fine_;
  Level lev_[kMaxLevels];
  hipStream_t s_ = nullptr;
  hipGraphExec_t gexec_[2] = {nullptr, nullptr};
  bool use_graphs_ = true;
  int threads_ = 0, rows_ = 0, order_ = 0;
  std::vector<void *> owned_;
};

// Checks of a multi-level configuration (mirrors hlbm.h).
int validate_levels(const hlbm_config &f, const hlbm_levels &lv, std::string *err) {
  if (lv.nlevels < 2 || lv.nlevels > HLBM_MAX_LEVELS) { *err = "nlevels must be 2 .. HLBM_MAX_LEVELS"; return HLBM_E_ARG; }
  if (lv.bc0 != HLBM_BC_PERIODIC_X_WALLS_Y && lv.bc0 != HLBM_BC_PERIODIC && lv.bc0 != HLBM_BC_PAPER) {
    *err = "unknown bc0";
    return HLBM_E_ARG;
  }
  int nx = lv.nx0, ny = lv.ny0;
  for (int l = 0; l < lv.nlevels - 1; ++l) {
    const int32_t *b = lv.box[l];
    if (nx < 3 || ny < 3 || b[0] < 2 || b[1] < 2 || b[2] > nx - 3 || b[3] > ny - 3 || b[2] - b[0] < 4 ||
        b[3] - b[1] < 4) {
      *err = "box of level " + std::to_string(l + 1) +
             " must lie two nodes inside level " + std::to_string(l) + " and span at least four cells";
      return HLBM_E_ARG;
    }
    nx = 2 * (b[2] - b[0]) + 1;
    ny = 2 * (b[3] - b[1]) + 1;
  }
  if (f.nx != nx || f.ny != ny) {
    *err = "finest level must be " + std::to_string(nx) + " x " + std::to_string(ny) + " nodes";
    return HLBM_E_ARG;
  }
  if (f.bc != HLBM_BC_RING) { *err = "the finest level takes bc HLBM_BC_RING"; return HLBM_E_ARG; }
  if (f.ckpt_every != 0) { *err = "a multi-level handle takes no checkpoints"; return HLBM_E_ARG; }
  return validate(f, err, true);
}

}  // namespace
}  // namespace mghlbm

struct hlbm {
  std::unique_ptr<mghlbm::CaseBase> c;
};

extern "C" {

int hlbm_create(const hlbm_config *cfg, int32_t ncases, hlbm_t **out) {
  using namespace mghlbm;
  if (out) *out = nullptr;
  if (!cfg || !out || ncases < 1) { g_create_error = "null argument or ncases < 1"; return HLBM_E_ARG; }
  std::string e;
  for (int i = 0; i < ncases; ++i) {
    int rc = validate(cfg[i], &e);
    if (rc != HLBM_OK) { g_create_error = (ncases > 1 ? "case " + std::to_string(i) + ": " : "") + e; return rc; }
    if (ncases > 1) {
      if (cfg[i].storage != cfg[0].storage) { g_create_error = "a batch needs one storage type"; return HLBM_E_ARG; }
      if (cfg[i].ckpt_every != 0) { g_create_error = "a batch takes no checkpoints"; return HLBM_E_ARG; }
      if (cfg[i].nux <= 0 || cfg[i].nuy <= 0) { g_create_error = "every batched case needs a grid"; return HLBM_E_ARG; }
    }
  }
  std::unique_ptr<CaseBase> c;
  int rc = HLBM_OK;
  try {
    if (ncases > 1) {
      if (cfg->storage == HLBM_FP64) {
        auto p = std::make_unique<Batch<double, double>>();
        rc = p->init(cfg, ncases);
        c = std::move(p);
      } else if (cfg->storage == HLBM_FP32) {
        auto p = std::make_unique<Batch<float, float>>();
        rc = p->init(cfg, ncases);
        c = std::move(p);
      } else {
        auto p = std::make_unique<Batch<__half, float>>();
        rc = p->init(cfg, ncases);
        c = std::move(p);
      }
    } else if (cfg->storage == HLBM_FP64) {
      auto p = std::make_unique<Case<double, double>>();
      rc = p->init(*cfg);
      c = std::move(p);
    } else if (cfg->storage == HLBM_FP32) {
      auto p = std::make_unique<Case<float, float>>();
      rc = p->init(*cfg);
      c = std::move(p);
    } else {
      auto p = std::make_unique<Case<__half, float>>();
      rc = p->init(*cfg);
      c = std::move(p);
    }
  } catch (const std::bad_alloc &) {
    g_create_error = "host allocation failed";
    return HLBM_E_NOMEM;
  }
  if (rc != HLBM_OK) {
    g_create_error = c->err;
    return rc == HLBM_E_HIP && g_create_error.find("out of memory") != std::string::npos ? HLBM_E_NOMEM : rc;
  }
  hlbm_t *h = new (std::nothrow) hlbm_t;
  if (!h) { g_create_error = "host allocation failed"; return HLBM_E_NOMEM; }
  h->c = std::move(c);
  *out = h;
  return HLBM_OK;
}

int hlbm_create_multilevel(const hlbm_config *fine, const hlbm_levels *lv, hlbm_t **out) {
  using namespace mghlbm;
  if (out) *out = nullptr;
  if (!fine || !lv || !out) { g_create_error = "null argument"; return HLBM_E_ARG; }
  std::string e;
  int rc = validate_levels(*fine, *lv, &e);
  if (rc != HLBM_OK) { g_create_error = e; return rc; }
  std::unique_ptr<CaseBase> c;
  try {
    if (fine->storage == HLBM_FP64) {
      auto p = std::make_unique<MultiLevel<double, double>>();
      rc = p->init(*fine, *lv);
      c = std::move(p);
    } else if (fine->storage == HLBM_FP32) {
      auto p = std::make_unique<MultiLevel<float, float>>();
      rc = p->init(*fine, *lv);
      c = std::move(p);
    } else {
      auto p = std::make_unique<MultiLevel<__half, float>>();
      rc = p->init(*fine, *lv);
      c = std::move(p);
    }
  } catch (const std::bad_alloc &) {
    g_create_error = "host allocation failed";
    return HLBM_E_NOMEM;
  }
  if (rc != HLBM_OK) {
    g_create_error = c->err;
    return rc == HLBM_E_HIP && g_create_error.find("out of memory") != std::string::npos ? HLBM_E_NOMEM : rc;
  }
  hlbm_t *h = new (std::nothrow) hlbm_t;
  if (!h) { g_create_error = "host allocation failed"; return HLBM_E_NOMEM; }
  h->c = std::move(c);
  *out = h;
  return HLBM_OK;
}

int hlbm_level_shape(hlbm_t *h, int32_t level, int32_t *nx, int32_t *ny, double *tau) {
  if (!h || !nx || !ny || !tau) return HLBM_E_ARG;
  int a = 0, b = 0;
  double t = 0.0;
  int rc = HLBM_E_STATE;
  if (auto *m64 = dynamic_cast<mghlbm::MultiLevel<double, double> *>(h->c.get())) rc = m64->shape(level, &a, &b, &t);
  else if (auto *m32 = dynamic_cast<mghlbm::MultiLevel<float, float> *>(h->c.get())) rc = m32->shape(level, &a, &b, &t);
  else if (auto *m16 = dynamic_cast<mghlbm::MultiLevel<__half, float> *>(h->c.get()))
    rc = m16->shape(level, &a, &b, &t);
  if (rc == HLBM_E_STATE) h->c->err = "not a multi-level handle";
  else if (rc != HLBM_OK) h->c->err = "level out of range";
  if (rc != HLBM_OK) return rc;
  *nx = a;
  *ny = b;
  *tau = t;
  return HLBM_OK;
}

int hlbm_create_mesh(const hlbm_config *cfg, int32_t nnode, const double *xy, const int32_t *node_type, int32_t ntri,
                     const int32_t *tri, hlbm_t **out) {
  using namespace mghlbm;
  if (out) *out = nullptr;
  if (!cfg || !xy || !node_type || !tri || !out) { g_create_error = "null argument"; return HLBM_E_ARG; }
  if (nnode < 3 || ntri < 1) { g_create_error = "mesh needs at least 3 nodes and 1 triangle"; return HLBM_E_ARG; }
  if (cfg->ckpt_every != 0) { g_create_error = "a mesh case takes no checkpoints (no adjoint)"; return HLBM_E_ARG; }
  // the lattice-level checks, then the grid's geometry from its bounding box
  hlbm_config lc = *cfg;
  lc.nux = lc.nuy = 0;
  std::string e;
  int rc = validate(lc, &e);
  if (rc != HLBM_OK) { g_create_error = e; return rc; }
  double x0 = xy[0], x1 = xy[0], y1 = xy[1];
  for (int p = 0; p < nnode; ++p) {
    if (!std::isfinite(xy[2 * p]) || !std::isfinite(xy[2 * p + 1])) { g_create_error = "mesh coordinate not finite"; return HLBM_E_ARG; }
    x0 = std::min(x0, xy[2 * p]);
    x1 = std::max(x1, xy[2 * p]);
    y1 = std::max(y1, xy[2 * p + 1]);
  }
  const Derived d = derive(*cfg, true);
  const bool body = cfg->b > 0.0 && !(cfg->flags & HLBM_FLAG_NO_BODY);
  if (!(1.0 / (double)d.n < 2.0 * d.tau_u)) { g_create_error = "grid sub-step violates Delta t_u < 2 tau_u"; return HLBM_E_ARG; }
  if (d.xc + x0 < 1.0 || d.xc + x1 > (double)cfg->nx - 2.0) { g_create_error = "grid leaves the lattice in x"; return HLBM_E_ARG; }
  if (cfg->bc != HLBM_BC_PERIODIC &&
      (d.yc - y1 - std::fabs(d.A) < 1.0 || d.yc + y1 + std::fabs(d.A) > (double)cfg->ny - 2.0)) {
    g_create_error = "grid motion leaves the lattice in y";
    return HLBM_E_ARG;
  }
  if (body && (!(cfg->thickness > 0.0) || 0.5 * cfg->b + 1.0 > -x0 - kMargin - 1.0 ||
               0.5 * cfg->b + 1.0 > x1 - kMargin - 1.0 || 0.5 * cfg->thickness + 1.0 > y1 - kMargin - 1.0)) {
    g_create_error = "lamina does not fit inside the fictitious rectangle";
    return HLBM_E_ARG;
  }
  if (!(std::fabs(d.A * d.omega) < 1.0)) { g_create_error = "lamina speed must stay below one lattice unit per step"; return HLBM_E_ARG; }
  const MeshInput mesh{nnode, xy, node_type, ntri, tri};
  std::unique_ptr<CaseBase> c;
  try {
    if (cfg->storage == HLBM_FP64) {
      auto p = std::make_unique<Case<double, double>>();
      rc = p->init(*cfg, true, nullptr, nullptr, &mesh);
      c = std::move(p);
    } else if (cfg->storage == HLBM_FP32) {
      auto p = std::make_unique<Case<float, float>>();
      rc = p->init(*cfg, true, nullptr, nullptr, &mesh);
      c = std::move(p);
    } else {
      auto p = std::make_unique<Case<__half, float>>();
      rc = p->init(*cfg, true, nullptr, nullptr, &mesh);
      c = std::move(p);
    }
  } catch (const std::bad_alloc &) {
    g_create_error = "host allocation failed";
    return HLBM_E_NOMEM;
  }
  if (rc != HLBM_OK) {
    g_create_error = c->err;
    return rc;
  }
  hlbm_t *h = new (std::nothrow) hlbm_t;
  if (!h) { g_create_error = "host allocation failed"; return HLBM_E_NOMEM; }
  h->c = std::move(c);
  *out = h;
  return HLBM_OK;
}

int hlbm_create_graded(const hlbm_config *cfg, const double *x_nodes, const double *y_nodes, hlbm_t **out) {
  using namespace mghlbm;
  if (out) *out = nullptr;
  if (!cfg || !x_nodes || !y_nodes || !out) { g_create_error = "null argument"; return HLBM_E_ARG; }
  if (cfg->nux <= 0 || cfg->nuy <= 0) { g_create_error = "a graded case needs a grid"; return HLBM_E_ARG; }
  std::string e;
  int rc = validate(*cfg, &e, false, x_nodes, y_nodes);
  if (rc != HLBM_OK) { g_create_error = e; return rc; }
  std::unique_ptr<CaseBase> c;
  try {
    if (cfg->storage == HLBM_FP64) {
      auto p = std::make_unique<Case<double, double>>();
      rc = p->init(*cfg, true, x_nodes, y_nodes);
      c = std::move(p);
    } else if (cfg->storage == HLBM_FP32) {
      auto p = std::make_unique<Case<float, float>>();
      rc = p->init(*cfg, true, x_nodes, y_nodes);
      c = std::move(p);
    } else {
      auto p = std::make_unique<Case<__half, float>>();
      rc = p->init(*cfg, true, x_nodes, y_nodes);
      c = std::move(p);
    }
  } catch (const std::bad_alloc &) {
    g_create_error = "host allocation failed";
    return HLBM_E_NOMEM;
  }
  if (rc != HLBM_OK) {
    g_create_error = c->err;
    return rc;
  }
  hlbm_t *h = new (std::nothrow) hlbm_t;
  if (!h) { g_create_error = "host allocation failed"; return HLBM_E_NOMEM; }
  h->c = std::move(c);
  *out = h;
  return HLBM_OK;
}

int hlbm_set_motion(hlbm_t *h, int32_t case_id, const hlbm_motion *m) {
  if (!h) return HLBM_E_ARG;
  h->c->drain();
  return h->c->set_motion(case_id, m);
}

int hlbm_set_deformation(hlbm_t *h, double B, double phi) {
  if (!h) return HLBM_E_ARG;
  h->c->drain();
  return h->c->set_deformation(B, phi);
}

int hlbm_step(hlbm_t *h, int64_t nsteps) {
  if (!h) return HLBM_E_ARG;
  return h->c->step(nsteps);
}

int hlbm_step_async(hlbm_t *h, int64_t nsteps) {
  if (!h) return HLBM_E_ARG;
  return h->c->step_async(nsteps);
}

int hlbm_sync(hlbm_t *h) {
  if (!h) return HLBM_E_ARG;
  return h->c->sync();
}

static mghlbm::CaseBase *pick(hlbm_t *h, int32_t case_id) {
  mghlbm::CaseBase *c = h->c->sub(case_id);
  if (!c) h->c->err = "case_id out of range";
  return c;
}

int hlbm_force(hlbm_t *h, int32_t case_id, double *hist_xy, int64_t cap, int64_t *n_out, double win_t0,
               double win_t1, double theta[2]) {
  if (!h || cap < 0) return HLBM_E_ARG;
  h->c->drain();
  mghlbm::CaseBase *c = pick(h, case_id);
  if (!c) return HLBM_E_ARG;
  const int rc = c->force(hist_xy, cap, n_out, win_t0, win_t1, theta);
  if (rc != HLBM_OK && c != h->c.get()) h->c->err = c->err;
  return rc;
}

int hlbm_adjoint(hlbm_t *h, int32_t case_id, const double *dJ_dF, int64_t n, double grad[3]) {
  if (!h) return HLBM_E_ARG;
  h->c->drain();
  if (h->c->sub(1)) return h->c->adjoint(dJ_dF, n, grad);  // a batch: unsupported
  if (case_id != 0) return HLBM_E_ARG;
  return h->c->adjoint(dJ_dF, n, grad);
}

int hlbm_get_state(hlbm_t *h, int32_t case_id, int32_t which, void *buf, size_t bytes) {
  if (!h || !buf) return HLBM_E_ARG;
  h->c->drain();
  mghlbm::CaseBase *c = pick(h, case_id);
  if (!c) return HLBM_E_ARG;
  const int rc = c->get_state(which, buf, bytes);
  if (rc != HLBM_OK && c != h->c.get()) h->c->err = c->err;
  return rc;
}

int hlbm_get_state_noalloc(hlbm_t *h, int32_t case_id, int32_t which, void *host_buf, size_t bytes) {
  if (!h || !host_buf) return HLBM_E_ARG;
  h->c->drain();
  mghlbm::CaseBase *c = pick(h, case_id);
  if (!c) return HLBM_E_ARG;
  const int rc = c->get_state_noalloc(which, host_buf, bytes);
  if (rc != HLBM_OK && c != h->c.get()) h->c->err = c->err;
  return rc;
}

int hlbm_set_state(hlbm_t *h, int32_t case_id, int32_t which, const void *buf, size_t bytes) {
  if (!h || !buf) return HLBM_E_ARG;
  h->c->drain();
  mghlbm::CaseBase *c = pick(h, case_id);
  if (!c) return HLBM_E_ARG;
  const int rc = c->set_state(which, buf, bytes);
  if (rc != HLBM_OK && c != h->c.get()) h->c->err = c->err;
  return rc;
}

int hlbm_info_get(hlbm_t *h, int32_t case_id, hlbm_info *out) {
  if (!h || !out) return HLBM_E_ARG;
  h->c->drain();
  mghlbm::CaseBase *c = pick(h, case_id);
  if (!c) return HLBM_E_ARG;
  const int rc = c->info(out);
  if (rc != HLBM_OK && c != h->c.get()) h->c->err = c->err;
  return rc;
}

int hlbm_tune(hlbm_t *h, int32_t trial_steps, hlbm_tuning *t) {
  if (!h) return HLBM_E_ARG;
  h->c->drain();
  return h->c->tune(trial_steps, t);
}

int hlbm_get_stencil(hlbm_t *h, int32_t kmax, int32_t *nbr, double *S, double *C) {
  if (!h || kmax <= 0) return HLBM_E_ARG;
  h->c->drain();
  return h->c->stencil(kmax, nbr, S, C);
}

int hlbm_timing(hlbm_t *h, int32_t on) {
  if (!h) return HLBM_E_ARG;
  h->c->drain();
  return h->c->timing(on);
}

int hlbm_timing_get(hlbm_t *h, int32_t kernel, double *total_ms, int64_t *count) {
  if (!h) return HLBM_E_ARG;
  h->c->drain();
  return h->c->timing_get(kernel, total_ms, count);
}

void hlbm_destroy(hlbm_t *h) { delete h; }

const char *hlbm_last_error(const hlbm_t *h) {
  if (!h) return mghlbm::g_create_error.c_str();
  return h->c->err.c_str();
}

}  // extern "C"
