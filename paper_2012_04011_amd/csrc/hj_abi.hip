// hj_abi.hip -- the C ABI (include/hj.h): validation, device buffers, the
// per-(v, theta) coefficient table, the CFL step and the step schedule.
// Every numerical step of the solve runs in the kernels of hj_kernels.hip.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <deque>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/hj.h"
#include "hj_internal.h"

namespace {

thread_local std::string g_last_error;

hj_status fail(hj_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HJ_HIP(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(e_ == hipErrorOutOfMemory ? HJ_ERR_OUT_OF_MEMORY : HJ_ERR_DEVICE,        \
                  "%s failed: %s", #call, hipGetErrorString(e_));                          \
  } while (0)

bool bit(uint32_t mask, int d) { return ((mask >> d) & 1u) != 0; }

// Steps the convergence mode enqueues between two looks at the stop flag.
constexpr int kConvergeChunk = 32;

}  // namespace

// ---- staging of hj_optimal_control_noalloc --------------------------------
// Host arrays given to hj_optimal_control_noalloc pass through this fixed
// device array: per state its (x, y, v, theta), its two controls and its
// value, 7 doubles (HJ_NOALLOC_MAX_STATES states, 3.5 MiB).  Each device
// holds its own copy until the process ends.  In host code the name is only
// a stand-in: host code reaches the memory through the address
// hipGetSymbolAddress gives on each device (noalloc_staging below).
static __device__ __align__(256) double scratch[(size_t)HJ_NOALLOC_MAX_STATES * 7];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
std::atomic<double *> g_scratch[kMaxDevices];

// The device address of `scratch` on device `dev`, which must be current:
// looked up once per device (hj_grid_create does it at set-up) and kept.
hj_status noalloc_staging(int dev, double **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(HJ_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
  double *p = g_scratch[dev].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    p = g_scratch[dev].load(std::memory_order_relaxed);
    if (!p) {
      void *addr = nullptr;
      hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !addr)
        return fail(HJ_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
      p = static_cast<double *>(addr);
      g_scratch[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return HJ_OK;
}

}  // namespace

struct hj_grid {
  hj_grid_desc g;
  hj_dynamics_desc dyn;
  hj_scheme_desc sch;
  hipStream_t stream = nullptr;
  int device = 0;
  int64_t npts = 0;
  size_t elem = 4;

  // device buffers (precision of the scheme)
  void *v0 = nullptr;   // target
  void *v = nullptr;    // current value V^n
  void *w1 = nullptr;   // RK stage value V^1
  void *w2 = nullptr;   // next value (swapped with v after a step)
  void *lut = nullptr;  // bx | by | ax | ay in the scheme's precision
  void *coef = nullptr;  // kp_x | km_x | kp_y | km_y (streaming kernel)
  void *th = nullptr;    // per v: alpha_th | sig_th | kp_th | km_th | sg_th (theta axis)
  // stage kernel: 2 = plane (LDS), 1 = streaming, 0 = generic
  int kernel = 0;
  int x_chunks = 1;
  int v_seg = 0, n_seg = 1;  // plane kernel: v rows per block, v segments
  // plane kernel's theta run length (runs of 3 hold whole planes only), and
  // a second one the autotuner times (0: none)
  int plane_run = 1, plane_run_alt = 0;
  // plane kernel: 0 = chunk mode (x_chunks), else the number of blocks that
  // share all row-planes (span mode, whole planes only)
  int span_blocks = 0;
  // plane kernel, chunk mode: y rows per block (2: two-row blocks, where
  // rows2_layout finds a layout for the run length)
  int plane_rows = 1;
  bool plane_ok = false, stream_ok = false;
  bool launch_fixed = false;   // kernel / chunks forced by the environment
  bool autotune_on = true, autotuned = false;
  void *v0xy = nullptr;        // target as an n0 x n1 table when constant over (v, theta)
  bool target_xy = false;
  double *lut64 = nullptr;  // ax | ay in FP64 for the CFL reduction
  double *amax_dev = nullptr;
  int32_t *flag_dev = nullptr;
  double *amax_host = nullptr;  // pinned
  int32_t *flag_host = nullptr;  // pinned

  // host-side constants of the Hamiltonian (see hj_internal.h)
  double bv = 0, bth = 0, av = 0, ath = 0, sig[4] = {0, 0, 0, 0}, sig_ball = 0;
  uint32_t ball_mask = 0;
  double h[4];
  std::vector<double> th_a, th_s;  // per v: alpha and input bound of the theta axis

  // convergence mode: the stop flag the stage kernels test (null otherwise)
  const int32_t *skip = nullptr;
  unsigned long long *conv_acc = nullptr;  // device: max |dV| of the step (bits)
  unsigned long long *eps_acc = nullptr;   // set: the plane kernel's last stage folds max |dV| into it
  int32_t *conv_state = nullptr;           // device: stopped, step count
  double *conv_eps = nullptr;              // device: eps of the last steps
  int32_t *conv_host = nullptr;            // pinned: state
  double *conv_eps_host = nullptr;         // pinned: eps log
  // derivative-range alpha (Algorithm 1): the state table (bx, by, ax, ay)
  // in FP64, device keys of the range, and the host copies of the tables
  std::vector<double> tab64;
  unsigned long long *range_keys = nullptr;
  unsigned long long *range_host = nullptr;  // pinned
  std::vector<double> up_lut, up_coef, up_th;
  std::vector<float> up32;
  // control queries: device copies of host states and results
  double *ctl_dev = nullptr;
  int64_t ctl_cap = 0;  // states

  bool has_target = false;
  bool dt_cached = false;
  double amax[4] = {0, 0, 0, 0};
  double dt_cfl = 0;  // +inf when nothing moves

  // step-loop timing: one (begin, end) event pair per timed solve, folded
  // into prof when read (no host synchronisation between solves)
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;  // pairs recorded since the last fold
  hj_profile prof = {0, 0, 0.0};

  // hj_solve_brt's time loop captured as a HIP graph and replayed (small
  // grids, where launch gaps are a large part of a step): one graph per
  // step count, step sizes, starting buffers and launch configuration
  struct SolveGraph {
    int64_t n;
    double dt, dt_last;
    void *v_in, *w2_in, *v_out, *w2_out;
    int kernel, x_chunks, plane_run, span_blocks, plane_rows;
    bool target_xy;
    const int32_t *skip;
    hipGraphExec_t exec;
  };
  std::vector<SolveGraph> graphs;  // most recent last
  hipStream_t cap_stream = nullptr;  // private stream the loop is captured on
  int graph_mode = -1;  // -1: by grid size, 0: never, 1: always (HJ_SOLVE_GRAPH)
};

namespace {

double spacing(const hj_grid_desc &g, int d) {
  if (bit(g.periodic_mask, d)) return (g.hi[d] - g.lo[d]) / g.n[d];
  return (g.hi[d] - g.lo[d]) / (g.n[d] - 1);
}

// Node coordinate x_i = lo + i h (the same expression everywhere; no fused
// multiply-add so that the table is reproducible on any host).
double node(const hj_grid_desc &g, int d, int i) {
#pragma clang fp contract(off)
  return g.lo[d] + i * spacing(g, d);
}

hj_status validate(const hj_grid_desc *g, const hj_dynamics_desc *dy, const hj_scheme_desc *s) {
  if (!g || !dy || !s) return fail(HJ_ERR_INVALID_ARG, "null descriptor");
  int64_t np = 1;
  for (int d = 0; d < 4; ++d) {
    if (g->n[d] < 3) return fail(HJ_ERR_INVALID_ARG, "grid axis %d has %d nodes (need >= 3)", d, g->n[d]);
    if (!isfinite(g->lo[d]) || !isfinite(g->hi[d]) || !(g->hi[d] > g->lo[d]))
      return fail(HJ_ERR_INVALID_ARG, "grid axis %d: need finite lo < hi", d);
    np *= g->n[d];
    if (np > INT32_MAX) return fail(HJ_ERR_INVALID_ARG, "grid has more than 2^31-1 nodes");
  }
  if (g->periodic_mask & ~0xFu) return fail(HJ_ERR_INVALID_ARG, "periodic_mask has bits above axis 3");
  if (dy->kind != HJ_DYN_CAR4D && dy->kind != HJ_DYN_DRIFT_INPUT && dy->kind != HJ_DYN_CAR4D_STEER)
    return fail(HJ_ERR_INVALID_ARG, "unknown dynamics kind %d", dy->kind);
  if (dy->kind == HJ_DYN_CAR4D_STEER &&
      (!isfinite(dy->steer_max) || dy->steer_max < 0 || dy->steer_max >= 1.5707963267948966 ||
       !isfinite(dy->wheelbase) || !(dy->wheelbase > 0)))
    return fail(HJ_ERR_INVALID_ARG, "steering car: need 0 <= steer_max < pi/2 and wheelbase > 0");
  double vals[] = {dy->a_max, dy->w_max, dy->d_max[0], dy->d_max[1], dy->in_speed};
  for (double x : vals)
    if (!isfinite(x) || x < 0) return fail(HJ_ERR_INVALID_ARG, "input bounds must be finite and >= 0");
  for (int d = 0; d < 4; ++d)
    if (!isfinite(dy->drift[d])) return fail(HJ_ERR_INVALID_ARG, "drift must be finite");
  if (dy->kind == HJ_DYN_DRIFT_INPUT) {
    if (dy->in_axes_mask & ~0xFu) return fail(HJ_ERR_INVALID_ARG, "in_axes_mask has bits above axis 3");
    if (dy->in_norm != HJ_NORM_BOX && dy->in_norm != HJ_NORM_BALL)
      return fail(HJ_ERR_INVALID_ARG, "unknown in_norm %d", dy->in_norm);
    if (dy->in_role != HJ_INPUT_MAXIMIZES && dy->in_role != HJ_INPUT_MINIMIZES)
      return fail(HJ_ERR_INVALID_ARG, "unknown in_role %d", dy->in_role);
  }
  if (s->deriv != HJ_UPWIND1 && s->deriv != HJ_ENO2) return fail(HJ_ERR_INVALID_ARG, "unknown deriv %d", s->deriv);
  if (s->integrator != HJ_EULER && s->integrator != HJ_TVD_RK2)
    return fail(HJ_ERR_INVALID_ARG, "unknown integrator %d", s->integrator);
  if (s->precision != HJ_F32 && s->precision != HJ_F64)
    return fail(HJ_ERR_INVALID_ARG, "unknown precision %d", s->precision);
  if (s->clamp != HJ_CLAMP_NONE && s->clamp != HJ_CLAMP_MIN_V0)
    return fail(HJ_ERR_INVALID_ARG, "unknown clamp %d", s->clamp);
  if (!(s->cfl > 0.0 && s->cfl <= 1.0)) return fail(HJ_ERR_INVALID_ARG, "cfl must lie in (0, 1]");
  if (s->alpha_mode != HJ_ALPHA_STATE && s->alpha_mode != HJ_ALPHA_DERIV_RANGE &&
      s->alpha_mode != HJ_ALPHA_DERIV_RANGE_ONESIDED)
    return fail(HJ_ERR_INVALID_ARG, "unknown alpha_mode %d", s->alpha_mode);
  return HJ_OK;
}

// Per-(v, theta) coefficient table in FP64 (bx, by, ax, ay) and the uniform
// constants.  Car: bx = v cos(theta), by = v sin(theta), alpha_x =
// |v cos(theta)| + d_x^max (the bound on |x'| over all inputs), alpha_y
// likewise; v' = a and theta' = w are pure inputs: sig = +a_max, +w_max
// (maximising control), -d_max on x, y (minimising disturbance).
void build_table(hj_grid *G, std::vector<double> &tab) {
#pragma clang fp contract(off)
  const hj_grid_desc &g = G->g;
  const hj_dynamics_desc &dy = G->dyn;
  int n2 = g.n[2], n3 = g.n[3];
  int64_t m = (int64_t)n2 * n3;
  tab.assign(4 * m, 0.0);
  for (int d = 0; d < 4; ++d) G->h[d] = spacing(g, d);
  G->th_a.assign(n2, 0.0);
  G->th_s.assign(n2, 0.0);
  if (dy.kind == HJ_DYN_CAR4D || dy.kind == HJ_DYN_CAR4D_STEER) {
    for (int k = 0; k < n2; ++k) {
      double v = node(g, 2, k);
      for (int l = 0; l < n3; ++l) {
        double th = node(g, 3, l);
        int64_t c = (int64_t)k * n3 + l;
        double bx = v * cos(th), by = v * sin(th);
        tab[c] = bx;
        tab[m + c] = by;
        tab[2 * m + c] = fabs(bx) + dy.d_max[0];
        tab[3 * m + c] = fabs(by) + dy.d_max[1];
      }
    }
    G->bv = 0;
    G->bth = 0;
    G->av = dy.a_max;
    G->sig[0] = -dy.d_max[0];
    G->sig[1] = -dy.d_max[1];
    G->sig[2] = dy.a_max;
    // theta' = w (|w| <= w_max), or v tan(delta) / L for the steering car:
    // a maximising input bounded by |v| tan(steer_max) / L at speed v
    for (int k = 0; k < n2; ++k) {
      double b = dy.kind == HJ_DYN_CAR4D ? dy.w_max : fabs(node(g, 2, k)) * tan(dy.steer_max) / dy.wheelbase;
      G->th_a[k] = b;
      G->th_s[k] = b;
    }
    G->sig_ball = 0;
    G->ball_mask = 0;
  } else {
    double s = dy.in_speed;
    double sgn = dy.in_role == HJ_INPUT_MAXIMIZES ? 1.0 : -1.0;
    double alpha[4];
    for (int d = 0; d < 4; ++d) alpha[d] = fabs(dy.drift[d]) + (bit(dy.in_axes_mask, d) ? s : 0.0);
    for (int64_t c = 0; c < m; ++c) {
      tab[c] = dy.drift[0];
      tab[m + c] = dy.drift[1];
      tab[2 * m + c] = alpha[0];
      tab[3 * m + c] = alpha[1];
    }
    G->bv = dy.drift[2];
    G->bth = dy.drift[3];
    G->av = alpha[2];
    for (int d = 0; d < 4; ++d)
      G->sig[d] = (dy.in_norm == HJ_NORM_BOX && bit(dy.in_axes_mask, d)) ? sgn * s : 0.0;
    for (int k = 0; k < n2; ++k) {
      G->th_a[k] = alpha[3];
      G->th_s[k] = G->sig[3];
    }
    G->sig_ball = dy.in_norm == HJ_NORM_BALL ? sgn * s : 0.0;
    G->ball_mask = dy.in_norm == HJ_NORM_BALL ? dy.in_axes_mask : 0u;
  }
  G->sig[3] = 0.0;  // the theta axis uses th_s (per v)
  G->ath = 0.0;     // alpha_theta^max over the grid's v nodes (CFL)
  for (int k = 0; k < n2; ++k)
    if (G->th_a[k] > G->ath) G->ath = G->th_a[k];
}

// Theta-axis table per v in FP64: alpha | sig | kp = (b + alpha) / (2h) |
// km = (b - alpha) / (2h) | sg = sig / (2h).
void build_theta(const hj_grid *G, std::vector<double> &th) {
  int n2 = G->g.n[2];
  th.assign(5 * (size_t)n2, 0.0);
  for (int k = 0; k < n2; ++k) {
    th[k] = G->th_a[k];
    th[n2 + k] = G->th_s[k];
    th[2 * n2 + k] = (G->bth + G->th_a[k]) / (2.0 * G->h[3]);
    th[3 * n2 + k] = (G->bth - G->th_a[k]) / (2.0 * G->h[3]);
    th[4 * n2 + k] = G->th_s[k] / (2.0 * G->h[3]);
  }
}

// Streaming-kernel coefficients from the FP64 table: per axis
// kp = (b + alpha) / (2h), km = (b - alpha) / (2h).
void build_coef(hj_grid *G, const std::vector<double> &tab, std::vector<double> &coef) {
  int64_t m = (int64_t)G->g.n[2] * G->g.n[3];
  coef.assign(4 * m, 0.0);
  for (int64_t c = 0; c < m; ++c) {
    double bx = tab[c], by = tab[m + c], ax = tab[2 * m + c], ay = tab[3 * m + c];
    coef[c] = (bx + ax) / (2.0 * G->h[0]);
    coef[m + c] = (bx - ax) / (2.0 * G->h[0]);
    coef[2 * m + c] = (by + ay) / (2.0 * G->h[1]);
    coef[3 * m + c] = (by - ay) / (2.0 * G->h[1]);
  }
}

// Number of x chunks a sweep is split into.  Streaming kernel: about four
// blocks of 256 threads per CU (256 CUs; 3 chunks on the 120x120x40x72 grid
// measured best among 1..10).  Plane kernel (one block per y row and chunk):
// about two blocks per CU.  Either way at least 8 planes per chunk (each
// chunk re-reads up to 4 planes to start its ring).
// x chunks of a handle without autotuning.  The plane kernel: about 3072
// waves in all (twelve per CU of 256), from ny blocks per chunk of
// block_waves waves each, at least 5 planes per chunk; the streaming kernel:
// about 1000 blocks, at least 8 planes per chunk.
int choose_x_chunks(int nx, int ny, int64_t slab_runs, bool plane, int block_waves) {
  const char *env = getenv("HJ_X_CHUNKS");
  if (env && atoi(env) > 0) {
    int c = atoi(env);
    return c > nx ? nx : c;
  }
  int64_t want, cap;
  if (plane) {
    const int64_t w = (int64_t)ny * (block_waves > 0 ? block_waves : 1);
    want = (3072 + w / 2) / w;
    cap = nx / 5;
  } else {
    int64_t bpc = (slab_runs + hj::kStreamBlock - 1) / hj::kStreamBlock;
    want = (1000 + bpc - 1) / bpc;
    cap = nx / 8;
  }
  if (cap < 1) cap = 1;
  int64_t c = want < cap ? want : cap;
  return c < 1 ? 1 : (int)c;
}

hipStream_t S(hj_grid *g) { return g->stream; }

template <typename T>
T *buf(void *p) {
  return static_cast<T *>(p);
}

void free_all(hj_grid *G) {
  void *ptrs[] = {G->v0,       G->v,           G->w1,       G->w2,       G->lut,      G->coef,
                  G->th,       G->v0xy,        G->lut64,    G->amax_dev, G->flag_dev, G->conv_acc,
                  G->conv_state, G->conv_eps, G->ctl_dev, G->range_keys};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (G->conv_host) (void)hipHostFree(G->conv_host);
  if (G->range_host) (void)hipHostFree(G->range_host);
  if (G->conv_eps_host) (void)hipHostFree(G->conv_eps_host);
  if (G->amax_host) (void)hipHostFree(G->amax_host);
  if (G->flag_host) (void)hipHostFree(G->flag_host);
  for (hipEvent_t e : G->ev_pool) (void)hipEventDestroy(e);
  G->ev_pool.clear();
  for (auto &e : G->graphs) (void)hipGraphExecDestroy(e.exec);
  G->graphs.clear();
  if (G->cap_stream) (void)hipStreamDestroy(G->cap_stream);
  G->cap_stream = nullptr;
}

// Fold the recorded event pairs into the profile (synchronises on them).
hj_status fold_events(hj_grid *G) {
  for (size_t i = 0; i < G->ev_used; ++i) {
    HJ_HIP(hipEventSynchronize(G->ev_pool[2 * i + 1]));
    float ms = 0;
    HJ_HIP(hipEventElapsedTime(&ms, G->ev_pool[2 * i], G->ev_pool[2 * i + 1]));
    G->prof.loop_ms += ms;
  }
  G->ev_used = 0;
  return HJ_OK;
}

// The next free (begin, end) pair, growing the pool as needed.
hj_status next_events(hj_grid *G, hipEvent_t *b, hipEvent_t *e) {
  while (G->ev_pool.size() < 2 * (G->ev_used + 1)) {
    hipEvent_t ev;
    HJ_HIP(hipEventCreate(&ev));
    G->ev_pool.push_back(ev);
  }
  *b = G->ev_pool[2 * G->ev_used];
  *e = G->ev_pool[2 * G->ev_used + 1];
  G->ev_used += 1;
  return HJ_OK;
}

hj_status check_handle(hj_grid *g) {
  if (!g) return fail(HJ_ERR_INVALID_ARG, "null handle");
  return HJ_OK;
}

hj_status check_array(const void *p, int32_t dtype, int32_t where) {
  if (!p) return fail(HJ_ERR_INVALID_ARG, "null array");
  if (dtype != HJ_F32 && dtype != HJ_F64) return fail(HJ_ERR_INVALID_ARG, "unknown dtype %d", dtype);
  if (where != HJ_HOST && where != HJ_DEVICE) return fail(HJ_ERR_INVALID_ARG, "unknown location %d", where);
  return HJ_OK;
}

hj_status set_device(hj_grid *G) {
  HJ_HIP(hipSetDevice(G->device));
  return HJ_OK;
}

// Is every value of a caller array finite?  Host arrays are scanned on the
// host; device arrays by a kernel (then one 4-byte read-back).
hj_status all_finite(hj_grid *G, const void *p, int32_t dtype, int32_t where, bool *ok) {
  int64_t n = G->npts;
  if (where == HJ_HOST) {
    *ok = true;
    if (dtype == HJ_F32) {
      const float *a = static_cast<const float *>(p);
      for (int64_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return *ok = false, HJ_OK;
    } else {
      const double *a = static_cast<const double *>(p);
      for (int64_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return *ok = false, HJ_OK;
    }
    return HJ_OK;
  }
  if (dtype == HJ_F32)
    HJ_HIP(hj::launch_nonfinite(static_cast<const float *>(p), n, G->flag_dev, S(G)));
  else
    HJ_HIP(hj::launch_nonfinite(static_cast<const double *>(p), n, G->flag_dev, S(G)));
  HJ_HIP(hipMemcpyAsync(G->flag_host, G->flag_dev, sizeof(int32_t), hipMemcpyDeviceToHost, S(G)));
  HJ_HIP(hipStreamSynchronize(S(G)));
  *ok = G->flag_host[0] == 0;
  return HJ_OK;
}

// Copy a caller array (any dtype / location) into the device buffer dst of
// the handle's precision.
hj_status import_array(hj_grid *G, void *dst, const void *src, int32_t dtype, int32_t where) {
  int64_t n = G->npts;
  bool same = (dtype == HJ_F32) == (G->elem == 4);
  if (where == HJ_DEVICE) {
    if (same) {
      HJ_HIP(hipMemcpyAsync(dst, src, n * G->elem, hipMemcpyDeviceToDevice, S(G)));
    } else if (G->elem == 4) {
      HJ_HIP(hj::launch_cast(buf<float>(dst), static_cast<const double *>(src), n, S(G)));
    } else {
      HJ_HIP(hj::launch_cast(buf<double>(dst), static_cast<const float *>(src), n, S(G)));
    }
    return HJ_OK;
  }
  if (same) {
    HJ_HIP(hipMemcpyAsync(dst, src, n * G->elem, hipMemcpyHostToDevice, S(G)));
    HJ_HIP(hipStreamSynchronize(S(G)));
    return HJ_OK;
  }
  // host array of the other precision: convert on the host, then copy
  if (G->elem == 4) {
    std::vector<float> tmp(n);
    const double *a = static_cast<const double *>(src);
    for (int64_t i = 0; i < n; ++i) tmp[i] = (float)a[i];
    HJ_HIP(hipMemcpyAsync(dst, tmp.data(), n * 4, hipMemcpyHostToDevice, S(G)));
    HJ_HIP(hipStreamSynchronize(S(G)));
  } else {
    std::vector<double> tmp(n);
    const float *a = static_cast<const float *>(src);
    for (int64_t i = 0; i < n; ++i) tmp[i] = (double)a[i];
    HJ_HIP(hipMemcpyAsync(dst, tmp.data(), n * 8, hipMemcpyHostToDevice, S(G)));
    HJ_HIP(hipStreamSynchronize(S(G)));
  }
  return HJ_OK;
}

hj_status export_array(hj_grid *G, const void *src, void *dst, int32_t dtype, int32_t where) {
  int64_t n = G->npts;
  bool same = (dtype == HJ_F32) == (G->elem == 4);
  if (where == HJ_DEVICE) {
    if (same) {
      HJ_HIP(hipMemcpyAsync(dst, src, n * G->elem, hipMemcpyDeviceToDevice, S(G)));
    } else if (G->elem == 4) {
      HJ_HIP(hj::launch_cast(static_cast<double *>(dst), static_cast<const float *>(src), n, S(G)));
    } else {
      HJ_HIP(hj::launch_cast(static_cast<float *>(dst), static_cast<const double *>(src), n, S(G)));
    }
    return HJ_OK;
  }
  if (same) {
    HJ_HIP(hipMemcpyAsync(dst, src, n * G->elem, hipMemcpyDeviceToHost, S(G)));
    HJ_HIP(hipStreamSynchronize(S(G)));
    return HJ_OK;
  }
  if (G->elem == 4) {
    std::vector<float> tmp(n);
    HJ_HIP(hipMemcpyAsync(tmp.data(), src, n * 4, hipMemcpyDeviceToHost, S(G)));
    HJ_HIP(hipStreamSynchronize(S(G)));
    double *o = static_cast<double *>(dst);
    for (int64_t i = 0; i < n; ++i) o[i] = tmp[i];
  } else {
    std::vector<double> tmp(n);
    HJ_HIP(hipMemcpyAsync(tmp.data(), src, n * 8, hipMemcpyDeviceToHost, S(G)));
    HJ_HIP(hipStreamSynchronize(S(G)));
    float *o = static_cast<float *>(dst);
    for (int64_t i = 0; i < n; ++i) o[i] = (float)tmp[i];
  }
  return HJ_OK;
}

// CFL step (Algorithm 1): alpha_d^max by the FP64 reduction kernel, then
// dt = cfl / sum_d(alpha_d^max / dx_d) on the host.  Cached per handle.
hj_status ensure_dt(hj_grid *G) {
  if (G->dt_cached) return HJ_OK;
  int64_t m = (int64_t)G->g.n[2] * G->g.n[3];
  HJ_HIP(hj::launch_alpha_max(G->lut64, G->lut64 + m, m, G->av, G->ath, G->amax_dev, S(G)));
  HJ_HIP(hipMemcpyAsync(G->amax_host, G->amax_dev, 4 * sizeof(double), hipMemcpyDeviceToHost, S(G)));
  HJ_HIP(hipStreamSynchronize(S(G)));
  double s = 0.0;
  for (int d = 0; d < 4; ++d) {
    G->amax[d] = G->amax_host[d];
    s += G->amax[d] / G->h[d];
  }
  G->dt_cfl = s == 0.0 ? INFINITY : G->sch.cfl / s;
  G->dt_cached = true;
  return HJ_OK;
}

// Fixed horizon: n = ceil(T / dt) steps of the CFL step dt, the last one
// shortened to T - (n - 1) dt (a zero CFL sum, i.e. nothing moves, makes one
// step of the whole horizon).  Needs ensure_dt.
void schedule(const hj_grid *G, double horizon, int64_t *n, double *dt, double *dt_last) {
  *dt = isinf(G->dt_cfl) ? horizon : G->dt_cfl;
  *n = 0;
  *dt_last = 0.0;
  if (horizon > 0.0) {
    *n = (int64_t)ceil(horizon / *dt);
    if (*n < 1) *n = 1;
    *dt_last = horizon - (double)(*n - 1) * *dt;
  }
}

template <typename T>
hj::StageArgs<T> stage_args(hj_grid *G) {
  hj::StageArgs<T> a;
  memset(&a, 0, sizeof a);
  const hj_grid_desc &g = G->g;
  for (int d = 0; d < 4; ++d) a.n[d] = g.n[d];
  a.st[3] = 1;
  a.st[2] = g.n[3];
  a.st[1] = (int64_t)g.n[2] * g.n[3];
  a.st[0] = (int64_t)g.n[1] * g.n[2] * g.n[3];
  a.periodic_mask = g.periodic_mask;
  for (int d = 0; d < 4; ++d) {
    a.inv_h[d] = (T)(1.0 / G->h[d]);
    a.sig[d] = (T)G->sig[d];
  }
  a.lut = buf<const T>(G->lut);
  a.th = buf<const T>(G->th);
  a.skip = G->skip;
  a.bv = (T)G->bv;
  a.bth = (T)G->bth;
  a.av = (T)G->av;
  a.ath = (T)G->ath;
  a.sig_ball = (T)G->sig_ball;
  a.ball_mask = G->ball_mask;
  a.npts = G->npts;
  return a;
}

// Two-row plane blocks (StreamArgs::rows = 2) for theta run `run`: each row's
// runs fill at most half a block in whole waves, so a row takes the whole
// (v, theta) plane or v segments of at least kPlaneMinSegRows rows (not with
// runs of 3 or ragged rows), and the LDS holds four plane buffers and four
// of the published neighbours.  False where no such layout exists.
bool rows2_layout(const hj_grid *G, int run, int *v_seg, int *n_seg) {
  const int ny = G->g.n[1], nv = G->g.n[2], nth = G->g.n[3];
  if (!G->plane_ok || run < 1 || ny < 2 || ny % 2 != 0 || G->ball_mask != 0) return false;
  const int rpr = (nth + run - 1) / run, sl = run == 3 ? 4 : run;
  const int per_row = (run == 3 ? hj::kPlaneMaxThreads3 : hj::kPlaneMaxThreads) / 2;  // a multiple of 64
  const int max_rows = per_row / rpr;
  if (max_rows < 1) return false;
  int ns = 1, vs = nv;
  if (nv > max_rows) {
    if (run == 3 || rpr * run != nth) return false;
    ns = (nv + max_rows - 1) / max_rows;
    vs = (nv + ns - 1) / ns;
    ns = (nv + vs - 1) / vs;
    if (vs < hj::kPlaneMinSegRows) return false;
  }
  const int64_t lrows = ns > 1 ? vs + 4 : nv;
  const int64_t lds = (4 * lrows + 4 * (int64_t)vs) * rpr * sl * G->elem;
  if (lds > hj::kPlaneMaxLdsBytes) return false;
  *v_seg = vs;
  *n_seg = ns;
  return true;
}

// The streaming description of the handle's grid for its own stage kernel
// (plane = the LDS plane kernel runs it, with the handle's plane run length
// or with plane_run, one of the handle's two; rows = 2: two-row blocks where
// they fit) or for the streaming tiles of the batched launches (plane =
// false).
template <typename T>
hj::StreamArgs<T> stream_args(hj_grid *G, bool plane, int plane_run = 0, int rows = 1) {
  hj::StreamArgs<T> a;
  memset(&a, 0, sizeof a);
  const hj_grid_desc &g = G->g;
  const int run = plane ? (plane_run ? plane_run : G->plane_run) : hj::run_length((int)sizeof(T), g.n[3]);
  int nseg = plane && run == 3 ? 1 : G->n_seg;  // runs of 3: whole planes
  int vseg = plane && run == 3 ? g.n[2] : G->v_seg;
  const bool two = plane && rows == 2 && rows2_layout(G, run, &vseg, &nseg);
  for (int d = 0; d < 4; ++d) a.n[d] = g.n[d];
  a.periodic_mask = g.periodic_mask;
  a.plane = g.n[1] * g.n[2] * g.n[3];
  a.row = g.n[2] * g.n[3];
  a.run = run;
  a.runs_per_row = (g.n[3] + run - 1) / run;  // the plane kernel's last run may overlap (ragged)
  a.slab_runs = g.n[1] * g.n[2] * a.runs_per_row;
  a.blocks_per_chunk = plane ? g.n[1] / (two ? 2 : 1) * nseg : (a.slab_runs + hj::kStreamBlock - 1) / hj::kStreamBlock;
  a.v_seg = vseg;
  a.n_seg = nseg;
  a.span = plane && nseg == 1 && !two ? G->span_blocks : 0;
  a.rows = two ? 2 : 1;
  a.n_chunks = G->x_chunks;
  a.chunk_len = (g.n[0] + a.n_chunks - 1) / a.n_chunks;
  a.n_chunks = (g.n[0] + a.chunk_len - 1) / a.chunk_len;
  a.coef = buf<const T>(G->coef);
  a.v0xy = G->target_xy ? buf<const T>(G->v0xy) : nullptr;
  // uniform v and theta coefficients: b = bv / bth, alpha = av / ath
  a.kp_v = (T)((G->bv + G->av) / (2.0 * G->h[2]));
  a.km_v = (T)((G->bv - G->av) / (2.0 * G->h[2]));
  a.coef_th = buf<const T>(G->th) + 2 * g.n[2];
  a.skip = G->skip;
  for (int d = 0; d < 4; ++d) {
    a.sg[d] = (T)(G->sig[d] / (2.0 * G->h[d]));
    a.half_inv_h[d] = (T)(1.0 / (2.0 * G->h[d]));
  }
  a.sig_ball = (T)G->sig_ball;
  a.ball_mask = G->ball_mask;
  return a;
}

template <typename T>
hj::StreamArgs<T> stream_args(hj_grid *G) {
  return stream_args<T>(G, G->kernel == 2, 0, G->plane_rows);
}

template <typename T>
hj_status launch_one_stage(hj_grid *G, const T *vs, const T *vn, T *out, int mode, int clamp, double dt,
                           bool last = false) {
  bool ball = G->ball_mask != 0;
  if (G->kernel > 0) {
    // the stage that folds eps (convergence mode) takes one-row plane blocks:
    // the runtime stage form spills registers in blocks of two rows
    const bool fold = last && G->kernel == 2 && G->eps_acc;
    hj::StreamArgs<T> a = fold ? stream_args<T>(G, true, 0, 1) : stream_args<T>(G);
    a.vs = vs;
    a.vn = vn;
    a.v0 = buf<const T>(G->v0);
    a.out = out;
    a.mode = mode;
    a.clamp = clamp;
    a.dt = (T)dt;
    if (fold) a.eps = G->eps_acc;
    if (G->kernel == 2)
      HJ_HIP(hj::launch_plane(a, G->sch.deriv, ball, S(G)));
    else
      HJ_HIP(hj::launch_stream(a, G->sch.deriv, ball, S(G)));
    return HJ_OK;
  }
  hj::StageArgs<T> a = stage_args<T>(G);
  a.vs = vs;
  a.vn = vn;
  a.v0 = buf<const T>(G->v0);
  a.out = out;
  a.mode = mode;
  a.clamp = clamp;
  a.dt = (T)dt;
  HJ_HIP(hj::launch_stage(a, G->sch.deriv, ball, S(G)));
  return HJ_OK;
}

// One full step of length dt: Euler (one stage) or TVD-RK2 (two stages),
// clamp fused into the last stage.  Swaps v and w2.
template <typename T>
hj_status enqueue_step(hj_grid *G, double dt, int64_t *launches) {
  hj_status st;
  int clamp = G->sch.clamp == HJ_CLAMP_MIN_V0;
  if (G->sch.integrator == HJ_EULER) {
    st = launch_one_stage<T>(G, buf<const T>(G->v), nullptr, buf<T>(G->w2), hj::kPlain, clamp, dt, true);
    if (st != HJ_OK) return st;
    *launches += 1;
  } else {
    st = launch_one_stage<T>(G, buf<const T>(G->v), nullptr, buf<T>(G->w1), hj::kPlain, 0, dt, false);
    if (st != HJ_OK) return st;
    st = launch_one_stage<T>(G, buf<const T>(G->w1), buf<const T>(G->v), buf<T>(G->w2), hj::kAverage, clamp, dt,
                             true);
    if (st != HJ_OK) return st;
    *launches += 2;
  }
  void *t = G->v;
  G->v = G->w2;
  G->w2 = t;
  return HJ_OK;
}

hj_status step_once(hj_grid *G, double dt, int64_t *launches) {
  if (G->elem == 4) return enqueue_step<float>(G, dt, launches);
  return enqueue_step<double>(G, dt, launches);
}

// ---- the solve loop as a HIP graph ----------------------------------------

constexpr size_t kSolveGraphs = 4;                      // graphs kept per handle
constexpr int64_t kSolveGraphMaxBytes = (int64_t)64 << 20;  // auto: arrays up to this size

bool use_solve_graph(hj_grid *G, int64_t n) {
  if (G->graph_mode < 0) {
    const char *env = getenv("HJ_SOLVE_GRAPH");
    G->graph_mode = env ? (atoi(env) != 0 ? 1 : 0) : 2;  // 2: by grid size
  }
  if (n < 2 || G->graph_mode == 0) return false;
  return G->graph_mode == 1 || G->npts * (int64_t)G->elem <= kSolveGraphMaxBytes;
}

// The n steps of a solve: replay the graph captured for this (n, dt,
// dt_last, starting buffers, launch configuration), capturing it first if
// needed.  The loop is captured on a private stream and launched on the
// handle's stream; the buffer roles end as the plain loop leaves them.
hj_status solve_graph(hj_grid *G, int64_t n, double dt, double dt_last, int64_t *launches) {
  const int per_step = G->sch.integrator == HJ_EULER ? 1 : 2;
  for (size_t i = 0; i < G->graphs.size(); ++i) {
    hj_grid::SolveGraph e = G->graphs[i];
    if (e.n == n && e.dt == dt && e.dt_last == dt_last && e.v_in == G->v && e.w2_in == G->w2 &&
        e.kernel == G->kernel && e.x_chunks == G->x_chunks && e.plane_run == G->plane_run &&
        e.span_blocks == G->span_blocks && e.plane_rows == G->plane_rows &&
        e.target_xy == G->target_xy && e.skip == G->skip) {
      HJ_HIP(hipGraphLaunch(e.exec, S(G)));
      G->v = e.v_out;
      G->w2 = e.w2_out;
      G->graphs.erase(G->graphs.begin() + i);
      G->graphs.push_back(e);
      *launches += per_step * n;
      return HJ_OK;
    }
  }
  if (!G->cap_stream) HJ_HIP(hipStreamCreateWithFlags(&G->cap_stream, hipStreamNonBlocking));
  hj_grid::SolveGraph e;
  e.n = n;
  e.dt = dt;
  e.dt_last = dt_last;
  e.v_in = G->v;
  e.w2_in = G->w2;
  e.kernel = G->kernel;
  e.x_chunks = G->x_chunks;
  e.plane_run = G->plane_run;
  e.span_blocks = G->span_blocks;
  e.plane_rows = G->plane_rows;
  e.target_xy = G->target_xy;
  e.skip = G->skip;
  e.exec = nullptr;
  hipStream_t user = G->stream;
  HJ_HIP(hipStreamBeginCapture(G->cap_stream, hipStreamCaptureModeThreadLocal));
  G->stream = G->cap_stream;
  int64_t captured = 0;
  hj_status st = HJ_OK;
  for (int64_t k = 0; k < n && st == HJ_OK; ++k) st = step_once(G, k + 1 < n ? dt : dt_last, &captured);
  G->stream = user;
  hipGraph_t graph = nullptr;
  hipError_t ce = hipStreamEndCapture(G->cap_stream, &graph);
  e.v_out = G->v;
  e.w2_out = G->w2;
  if (st != HJ_OK || ce != hipSuccess) {
    G->v = e.v_in;  // nothing ran: the buffer roles stay as they were
    G->w2 = e.w2_in;
    if (graph) (void)hipGraphDestroy(graph);
    if (st != HJ_OK) return st;
    return fail(HJ_ERR_DEVICE, "HIP error %d (%s) capturing the solve loop", (int)ce, hipGetErrorString(ce));
  }
  hipError_t ie = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    G->v = e.v_in;
    G->w2 = e.w2_in;
    return fail(HJ_ERR_DEVICE, "HIP error %d (%s) instantiating the solve loop", (int)ie, hipGetErrorString(ie));
  }
  if (G->graphs.size() >= kSolveGraphs) {
    (void)hipGraphExecDestroy(G->graphs.front().exec);
    G->graphs.erase(G->graphs.begin());
  }
  G->graphs.push_back(e);
  HJ_HIP(hipGraphLaunch(e.exec, S(G)));
  *launches += captured;
  return HJ_OK;
}

// ---- Algorithm 1's derivative-range alpha ----------------------------------

double key_to_double(unsigned long long k) {
  unsigned long long b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
  double x;
  memcpy(&x, &b, sizeof x);
  return x;
}

// A box-bounded input that is +dir*bound where its gradient component is
// >= 0 and -dir*bound where it is < 0: the largest |b + input| over the
// gradient range [lo, hi].
double range_box_alpha(double b, double bound, int dir, double lo, double hi) {
  double best = 0.0;
  if (hi >= 0.0) best = fabs(b + dir * bound);
  if (lo < 0.0) {
    double c = fabs(b - dir * bound);
    if (c > best) best = c;
  }
  return best;
}

// Extremes of p_d / |p_S| over the gradient box (0 where p_S = 0).
void range_ball_ratio(const double lo[4], const double hi[4], uint32_t mask, int d, double *gmin, double *gmax) {
  double near2 = 0.0, far2 = 0.0;
  for (int e = 0; e < 4; ++e) {
    if (e == d || !bit(mask, e)) continue;
    double a = lo[e] * lo[e], b = hi[e] * hi[e];
    far2 += a > b ? a : b;
    if (lo[e] > 0.0 || hi[e] < 0.0) near2 += a < b ? a : b;
  }
  double M = hi[d], m = lo[d];
  *gmax = M > 0.0 ? M / sqrt(M * M + near2) : (M < 0.0 ? M / sqrt(M * M + far2) : 0.0);
  *gmin = m < 0.0 ? m / sqrt(m * m + near2) : (m > 0.0 ? m / sqrt(m * m + far2) : 0.0);
}

template <typename T>
hj_status upload_tables(hj_grid *G, void *dst, const std::vector<double> &src) {
  if (G->elem == 8) {
    HJ_HIP(hipMemcpyAsync(dst, src.data(), src.size() * 8, hipMemcpyHostToDevice, S(G)));
  } else {
    // the float staging copy of each table lives until the next range update
    // (which synchronises first)
    size_t off = G->up32.size();
    G->up32.resize(off + src.size());
    for (size_t i = 0; i < src.size(); ++i) G->up32[off + i] = (float)src[i];
    HJ_HIP(hipMemcpyAsync(dst, G->up32.data() + off, src.size() * 4, hipMemcpyHostToDevice, S(G)));
  }
  return HJ_OK;
}

// Derivative range of the current V on the device, Algorithm 1's alpha on
// the host, the stage tables rewritten with it; *dt_allowed = cfl / sum_d
// alpha_d^max / dx_d (+inf when nothing moves).  Synchronises.
hj_status range_alpha_update(hj_grid *G, double *dt_allowed) {
  hj_status st0 = ensure_dt(G);  // caches the state-bound step before av is rewritten below
  if (st0 != HJ_OK) return st0;
  if (!G->range_keys) {
    HJ_HIP(hipMalloc((void **)&G->range_keys, 8 * hj::kRangeSlots * sizeof(unsigned long long)));
    HJ_HIP(hipHostMalloc((void **)&G->range_host, 8 * hj::kRangeSlots * sizeof(unsigned long long), 0));
  }
  // the plane kernel's own traversal where it runs the grid, else the
  // one-thread-per-column pass
  const int32_t onesided = G->sch.alpha_mode == HJ_ALPHA_DERIV_RANGE_ONESIDED ? 1 : 0;
  if (G->kernel == 2 && G->elem == 4) {
    hj::StreamArgs<float> a = stream_args<float>(G, true, 0, 1);  // the range pass takes one-row blocks
    a.vs = buf<const float>(G->v);
    a.range = G->range_keys;
    a.range_onesided = onesided;
    HJ_HIP(hj::launch_plane_range(a, G->sch.deriv, S(G)));
  } else if (G->kernel == 2) {
    hj::StreamArgs<double> a = stream_args<double>(G, true, 0, 1);
    a.vs = buf<const double>(G->v);
    a.range = G->range_keys;
    a.range_onesided = onesided;
    HJ_HIP(hj::launch_plane_range(a, G->sch.deriv, S(G)));
  } else if (G->elem == 4) {
    hj::StageArgs<float> a = stage_args<float>(G);
    a.vs = buf<const float>(G->v);
    a.range_onesided = onesided;
    HJ_HIP(hj::launch_deriv_range(a, G->sch.deriv, G->range_keys, S(G)));
  } else {
    hj::StageArgs<double> a = stage_args<double>(G);
    a.vs = buf<const double>(G->v);
    a.range_onesided = onesided;
    HJ_HIP(hj::launch_deriv_range(a, G->sch.deriv, G->range_keys, S(G)));
  }
  HJ_HIP(hipMemcpyAsync(G->range_host, G->range_keys, 8 * hj::kRangeSlots * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, S(G)));
  HJ_HIP(hipStreamSynchronize(S(G)));  // also retires the previous update's uploads
  double lo[4], hi[4];
  for (int d = 0; d < 4; ++d) {
    unsigned long long kl = G->range_host[d], kh = G->range_host[4 + d];
    for (int k = 1; k < hj::kRangeSlots; ++k) {
      kl = std::min(kl, G->range_host[8 * k + d]);
      kh = std::max(kh, G->range_host[8 * k + 4 + d]);
    }
    lo[d] = key_to_double(kl);
    hi[d] = key_to_double(kh);
  }
  const hj_dynamics_desc &dy = G->dyn;
  const int n2 = G->g.n[2], n3 = G->g.n[3];
  const int64_t m = (int64_t)n2 * n3;
  const std::vector<double> &tab = G->tab64;
  G->up_lut.assign(tab.begin(), tab.end());
  double amax[4] = {0, 0, 0, 0};
  std::vector<double> ath(n2);
  if (dy.kind == HJ_DYN_CAR4D || dy.kind == HJ_DYN_CAR4D_STEER) {
    for (int64_t c = 0; c < m; ++c) {  // the disturbance is -d_max where p >= 0
      G->up_lut[2 * m + c] = range_box_alpha(tab[c], dy.d_max[0], -1, lo[0], hi[0]);
      G->up_lut[3 * m + c] = range_box_alpha(tab[m + c], dy.d_max[1], -1, lo[1], hi[1]);
    }
    G->av = range_box_alpha(0.0, dy.a_max, +1, lo[2], hi[2]);
    for (int k = 0; k < n2; ++k) ath[k] = range_box_alpha(0.0, G->th_s[k], +1, lo[3], hi[3]);
  } else {
    const int dir = dy.in_role == HJ_INPUT_MAXIMIZES ? 1 : -1;
    double al[4];
    for (int d = 0; d < 4; ++d) {
      if (!bit(dy.in_axes_mask, d)) {
        al[d] = fabs(dy.drift[d]);
      } else if (dy.in_norm == HJ_NORM_BOX) {
        al[d] = range_box_alpha(dy.drift[d], dy.in_speed, dir, lo[d], hi[d]);
      } else {
        double gmin, gmax;
        range_ball_ratio(lo, hi, dy.in_axes_mask, d, &gmin, &gmax);
        double a1 = fabs(dy.drift[d] + dir * dy.in_speed * gmax), a2 = fabs(dy.drift[d] + dir * dy.in_speed * gmin);
        al[d] = a1 > a2 ? a1 : a2;
      }
    }
    for (int64_t c = 0; c < m; ++c) {
      G->up_lut[2 * m + c] = al[0];
      G->up_lut[3 * m + c] = al[1];
    }
    G->av = al[2];
    for (int k = 0; k < n2; ++k) ath[k] = al[3];
  }
  for (int64_t c = 0; c < m; ++c) {
    if (G->up_lut[2 * m + c] > amax[0]) amax[0] = G->up_lut[2 * m + c];
    if (G->up_lut[3 * m + c] > amax[1]) amax[1] = G->up_lut[3 * m + c];
  }
  amax[2] = G->av;
  for (int k = 0; k < n2; ++k)
    if (ath[k] > amax[3]) amax[3] = ath[k];
  // the stage tables with this alpha (the Hamiltonian's own terms unchanged)
  build_coef(G, G->up_lut, G->up_coef);
  std::vector<double> keep_a = G->th_a;
  G->th_a = ath;
  build_theta(G, G->up_th);
  G->th_a = keep_a;
  G->up32.clear();
  G->up32.reserve(G->up_lut.size() + G->up_coef.size() + G->up_th.size());
  hj_status st;
  if ((st = upload_tables<double>(G, G->lut, G->up_lut)) != HJ_OK) return st;
  if ((st = upload_tables<double>(G, G->coef, G->up_coef)) != HJ_OK) return st;
  if ((st = upload_tables<double>(G, G->th, G->up_th)) != HJ_OK) return st;
  double sum = 0.0;
  for (int d = 0; d < 4; ++d) sum += amax[d] / G->h[d];
  *dt_allowed = sum == 0.0 ? INFINITY : G->sch.cfl / sum;
  (void)n3;
  return HJ_OK;
}

hj_status reset_value(hj_grid *G) {
  HJ_HIP(hipMemcpyAsync(G->v, G->v0, G->npts * G->elem, hipMemcpyDeviceToDevice, S(G)));
  return HJ_OK;
}

// Time `reps` full steps of the current configuration on scratch buffers:
// stage 1 reads V and writes w1, stage 2 reads w1 and V and writes w2 (no
// swap), so V is left as it was.  Returns milliseconds per step.
template <typename T>
hj_status time_config(hj_grid *G, int reps, hipEvent_t e0, hipEvent_t e1, float *ms) {
  hj_status st;
  int clamp = G->sch.clamp == HJ_CLAMP_MIN_V0;
  const T *v = buf<const T>(G->v);
  auto one = [&]() -> hj_status {
    if (G->sch.integrator == HJ_EULER)
      return launch_one_stage<T>(G, v, nullptr, buf<T>(G->w2), hj::kPlain, clamp, G->dt_cfl);
    hj_status s1 = launch_one_stage<T>(G, v, nullptr, buf<T>(G->w1), hj::kPlain, 0, G->dt_cfl);
    if (s1 != HJ_OK) return s1;
    return launch_one_stage<T>(G, buf<const T>(G->w1), v, buf<T>(G->w2), hj::kAverage, clamp, G->dt_cfl);
  };
  if ((st = one()) != HJ_OK) return st;  // warm-up
  HJ_HIP(hipEventRecord(e0, S(G)));
  for (int i = 0; i < reps; ++i)
    if ((st = one()) != HJ_OK) return st;
  HJ_HIP(hipEventRecord(e1, S(G)));
  HJ_HIP(hipEventSynchronize(e1));
  HJ_HIP(hipEventElapsedTime(ms, e0, e1));
  *ms /= reps;
  return HJ_OK;
}

// Compute units of a device (0 if unknown), looked up once per device.
int device_cus(int dev) {
  static std::mutex mu;
  static std::map<int, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int n = 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) n = 0;
  cache[dev] = n;
  return n;
}

hj_status autotune(hj_grid *G) {
  hj_status st;
  if ((st = ensure_dt(G)) != HJ_OK) return st;
  if (isinf(G->dt_cfl) || (!G->plane_ok && !G->stream_ok)) {
    G->autotuned = true;
    return HJ_OK;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HJ_HIP(hipEventCreate(&e0));
  HJ_HIP(hipEventCreate(&e1));
  int best_k = G->kernel, best_c = G->x_chunks, best_r = G->plane_run, best_s = G->span_blocks;
  int best_w = G->plane_rows;
  const int cus = device_cus(G->device);
  struct Cand {
    int k, c, r, s, w;
    float ms;
  };
  std::vector<Cand> cands;
  // (kernel, plane run, rows per block) candidates: the plane kernel with its
  // run length and the alternative, each with one-row and (where they fit)
  // two-row blocks, then the streaming kernel; HJ_PLANE_ROWS=1|2 keeps one
  const char *rows_env = getenv("HJ_PLANE_ROWS");
  const int rows_only = rows_env ? atoi(rows_env) : 0;
  int kernels[5] = {2, 2, 2, 2, 1}, runs[5] = {G->plane_run, G->plane_run, G->plane_run_alt, G->plane_run_alt, G->plane_run};
  int rowsv[5] = {1, 2, 1, 2, 1};
  int cap = G->g.n[0] / 4 > 1 ? G->g.n[0] / 4 : 1;
  for (int kk = 0; kk < 5 && st == HJ_OK; ++kk) {
    int k = kernels[kk];
    if ((k == 2 && !G->plane_ok) || (k == 1 && !G->stream_ok) || runs[kk] == 0) continue;
    int vs_unused, ns_unused;
    if (k == 2 && rowsv[kk] == 2 && !rows2_layout(G, runs[kk], &vs_unused, &ns_unused)) continue;
    if (k == 2 && rows_only && rowsv[kk] != rows_only) continue;
    // chunk modes 1 .. 8, 10, 12, 16 (at least 4 planes each), then (plane
    // kernel, whole planes, one-row blocks) blocks that share all row-planes:
    // one or two per CU
    const bool whole = runs[kk] == 3 || G->n_seg == 1;
    const int nspan = k == 2 && whole && rowsv[kk] == 1 && cus > 0 ? 2 : 0;
    static const int kChunks[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 16};
    const int nchunk = (int)(sizeof kChunks / sizeof kChunks[0]);
    for (int ci = 0; ci < nchunk + nspan; ++ci) {
      const bool span = ci >= nchunk;
      const int c = span ? 0 : kChunks[ci];
      if (!span && c > cap) continue;
      G->kernel = k;
      G->x_chunks = span ? G->x_chunks : c;
      G->span_blocks = span ? (ci - nchunk + 1) * cus : 0;
      G->plane_run = runs[kk];
      G->plane_rows = rowsv[kk];
      float ms = 0;
      st = G->elem == 4 ? time_config<float>(G, 5, e0, e1, &ms) : time_config<double>(G, 5, e0, e1, &ms);
      if (st != HJ_OK) break;
      if (getenv("HJ_AUTOTUNE_VERBOSE"))
        fprintf(stderr, "hj_autotune: kernel %d run %d rows %d chunks %d span %d: %.1f us per step\n", k, runs[kk],
                rowsv[kk], G->x_chunks, G->span_blocks, ms * 1e3);
      cands.push_back({k, G->x_chunks, runs[kk], G->span_blocks, rowsv[kk], ms});
    }
  }
  // the three fastest again, in three alternating rounds: one short timing
  // can rank candidates a few per cent apart by the noise of its launches
  std::stable_sort(cands.begin(), cands.end(), [](const Cand &x, const Cand &y) { return x.ms < y.ms; });
  if (cands.size() > 3) cands.resize(3);
  std::vector<float> total(cands.size(), 0.0f);
  for (int round = 0; round < 3 && st == HJ_OK && cands.size() > 1; ++round)
    for (size_t i = 0; i < cands.size() && st == HJ_OK; ++i) {
      G->kernel = cands[i].k;
      G->x_chunks = cands[i].c;
      G->plane_run = cands[i].r;
      G->span_blocks = cands[i].s;
      G->plane_rows = cands[i].w;
      float ms = 0;
      st = G->elem == 4 ? time_config<float>(G, 5, e0, e1, &ms) : time_config<double>(G, 5, e0, e1, &ms);
      total[i] += ms;
    }
  if (!cands.empty()) {
    size_t b = 0;
    for (size_t i = 1; i < cands.size(); ++i)
      if (total[i] < total[b]) b = i;
    if (getenv("HJ_AUTOTUNE_VERBOSE") && cands.size() > 1)
      fprintf(stderr, "hj_autotune: kept kernel %d run %d rows %d chunks %d span %d (%.1f us per step over 3 rounds)\n",
              cands[b].k, cands[b].r, cands[b].w, cands[b].c, cands[b].s, total[b] / 3 * 1e3);
    best_k = cands[b].k;
    best_c = cands[b].c;
    best_r = cands[b].r;
    best_s = cands[b].s;
    best_w = cands[b].w;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  G->kernel = best_k;
  G->x_chunks = best_c;
  G->plane_run = best_r;
  G->span_blocks = best_s;
  G->plane_rows = best_w;
  if (st == HJ_OK) G->autotuned = true;
  return st;
}

}  // namespace

extern "C" {

const char *hj_last_error(void) { return g_last_error.c_str(); }

const char *hj_version(void) { return "hjreach-gfx950 0.1"; }

hj_status hj_grid_create(const hj_grid_desc *grid, const hj_dynamics_desc *dyn, const hj_scheme_desc *scheme,
                         void *hip_stream, hj_grid **out) {
  if (!out) return fail(HJ_ERR_INVALID_ARG, "null output handle pointer");
  *out = nullptr;
  hj_status st = validate(grid, dyn, scheme);
  if (st != HJ_OK) return st;
  hj_grid *G = new (std::nothrow) hj_grid;
  if (!G) return fail(HJ_ERR_OUT_OF_MEMORY, "host allocation failed");
  G->g = *grid;
  G->dyn = *dyn;
  G->sch = *scheme;
  G->stream = static_cast<hipStream_t>(hip_stream);
  G->npts = (int64_t)grid->n[0] * grid->n[1] * grid->n[2] * grid->n[3];
  G->elem = scheme->precision == HJ_F32 ? 4 : 8;
  std::vector<double> tab, coef, th;
  build_table(G, tab);
  build_coef(G, tab, coef);
  build_theta(G, th);
  if (scheme->alpha_mode != HJ_ALPHA_STATE) G->tab64 = tab;
  int64_t m = (int64_t)grid->n[2] * grid->n[3];
  {
    int run = hj::run_length(G->elem, grid->n[3]);
    // theta periodic; 32-bit byte offsets (buffer addressing) need each
    // array below 4 GiB
    bool stream_ok = bit(grid->periodic_mask, 3) && G->npts * (int64_t)G->elem < ((int64_t)1 << 32);
    const int nv = grid->n[2], nth = grid->n[3];
    const char *vseg_env = getenv("HJ_PLANE_VSEG");
    // SIMD time per plane of a run length (see the runs-of-3 choice below)
    auto cost = [&](int r, int64_t runs_r) {
      const int64_t waves = (runs_r + 63) / 64;
      return (double)(waves >= 8 ? 4 * ((waves + 3) / 4) : waves) * (51.0 * r + 15.0);
    };
    // An odd N_theta gives runs of one theta node, an even one not divisible
    // by 4 runs of two in FP32; the plane kernel takes runs of 4 (FP32; 2 in
    // FP64) instead -- for runs of two where they cost less -- the last run
    // of a row shifted back to end at the row's end (it repeats nodes of the
    // run before it), where the whole plane fits one block
    {
      const int rr = G->elem == 4 ? 4 : 2;
      const int64_t rruns = (int64_t)nv * ((nth + rr - 1) / rr);
      const bool fits = nth >= 2 * rr && !vseg_env && rruns <= hj::kPlaneMaxThreads &&
                        2 * rruns * rr * (int64_t)G->elem <= hj::kPlaneMaxLdsBytes;
      if (fits && (run == 1 || (run == 2 && rr == 4 && cost(4, rruns) < cost(2, (int64_t)nv * (nth / 2)))))
        run = rr;
    }
    const int rpr = (nth + run - 1) / run;
    int64_t plane_runs = (int64_t)nv * rpr;
    // The plane kernel holds the whole (v, theta) plane in one block when it
    // has at most kPlaneMaxThreads runs, else the fewest v segments that fit
    // (HJ_PLANE_VSEG caps the rows per block, to exercise the split).
    int max_rows = hj::kPlaneMaxThreads / rpr;
    if (vseg_env && atoi(vseg_env) > 0 && atoi(vseg_env) < max_rows) max_rows = atoi(vseg_env);
    int n_seg = 1, v_seg = nv;
    if (max_rows > 0 && nv > max_rows) {
      n_seg = (nv + max_rows - 1) / max_rows;
      v_seg = (nv + n_seg - 1) / n_seg;
      n_seg = (nv + v_seg - 1) / v_seg;
    }
    const int64_t lds_rows = n_seg > 1 ? v_seg + 4 : nv;
    bool plane_ok = stream_ok && max_rows > 0 && (n_seg == 1 || v_seg >= hj::kPlaneMinSegRows) &&
                    2 * lds_rows * rpr * run * (int64_t)G->elem <= hj::kPlaneMaxLdsBytes;
    G->v_seg = v_seg;
    G->n_seg = plane_ok ? n_seg : 1;
    G->plane_run = run;
    // Runs of 3 theta nodes (FP32): a whole plane in one block of up to
    // kPlaneMaxThreads3 runs, each run in a 4-element LDS slot.  Taken where
    // it costs less SIMD time per plane: a thread's plane costs about
    // 51 R + 15 instructions (R nodes' four axes and update, its run's theta
    // halo, per-thread overhead), idle lanes of the last wave cost the same,
    // and a block of 8 or more waves (alone on its CU) takes as long as its
    // busiest SIMD (waves / 4, rounded up), since a barrier ends each plane.
    const int64_t runs3 = (int64_t)nv * (grid->n[3] / 3);
    const bool fit3 = G->elem == 4 && grid->n[3] % 3 == 0 && stream_ok && !vseg_env &&
                      runs3 <= hj::kPlaneMaxThreads3 && 2 * runs3 * 4 * 4 <= hj::kPlaneMaxLdsBytes;
    const bool plane_ok_default = plane_ok;
    if (fit3) {
      const bool three_better = !plane_ok || n_seg > 1 || cost(3, runs3) < cost(run, plane_runs);
      if (!plane_ok) {  // runs of 3 make a whole plane fit
        plane_ok = true;
        G->n_seg = 1;
        G->v_seg = nv;
      }
      G->plane_run = three_better ? 3 : run;
      G->plane_run_alt = three_better ? (plane_ok_default ? run : 0) : 3;
    }
    const char *prun = getenv("HJ_PLANE_RUN");
    if (prun && fit3 && atoi(prun) == 3) {
      G->plane_run = 3;
      G->plane_run_alt = 0;
    } else if (prun && atoi(prun) == run && plane_ok_default) {
      G->plane_run = run;
      G->plane_run_alt = 0;
    }
    G->plane_ok = plane_ok;
    G->stream_ok = stream_ok;
    G->kernel = plane_ok ? 2 : (stream_ok ? 1 : 0);
    const char *force = getenv("HJ_STAGE_KERNEL");
    if (force) {
      if (!strcmp(force, "generic")) G->kernel = 0;
      if (!strcmp(force, "stream") && stream_ok) G->kernel = 1;
      G->launch_fixed = true;
    }
    if (getenv("HJ_X_CHUNKS")) G->launch_fixed = true;
    // two-row plane blocks where they fit (HJ_PLANE_ROWS=2; else the
    // autotuner's choice)
    const char *rows_env = getenv("HJ_PLANE_ROWS");
    int vs2 = 0, ns2 = 0;
    if (rows_env && atoi(rows_env) == 2 && G->kernel == 2 && rows2_layout(G, G->plane_run, &vs2, &ns2))
      G->plane_rows = 2;
    const char *span_env = getenv("HJ_PLANE_SPAN");  // blocks sharing all row-planes (plane kernel, whole planes)
    if (span_env && atoi(span_env) > 0) {
      G->span_blocks = atoi(span_env);
      G->launch_fixed = true;
    }
    int64_t slab_runs = (int64_t)grid->n[1] * plane_runs;
    const int bseg = G->plane_run == 3 ? 1 : G->n_seg;
    const int64_t block_runs =
        (int64_t)(bseg > 1 ? G->v_seg : nv) * ((grid->n[3] + G->plane_run - 1) / G->plane_run);
    G->x_chunks = choose_x_chunks(grid->n[0], grid->n[1] * bseg, slab_runs, G->kernel == 2,
                                  (int)((block_runs + 63) / 64));
  }
  hipError_t e = hipGetDevice(&G->device);
  if (e == hipSuccess) {
    // set-up of this device's staging for hj_optimal_control_noalloc (a
    // failure here is reported by that call, which looks again)
    double *unused = nullptr;
    (void)noalloc_staging(G->device, &unused);
    g_last_error.clear();
  }
  size_t bytes = G->npts * G->elem;
  bool rk2 = scheme->integrator == HJ_TVD_RK2;
  if (e == hipSuccess) e = hipMalloc(&G->v0, bytes);
  if (e == hipSuccess) e = hipMalloc(&G->v, bytes);
  if (e == hipSuccess) e = hipMalloc(&G->w2, bytes);
  if (e == hipSuccess && rk2) e = hipMalloc(&G->w1, bytes);
  if (e == hipSuccess) e = hipMalloc(&G->lut, 4 * m * G->elem);
  if (e == hipSuccess) e = hipMalloc(&G->coef, 4 * m * G->elem);
  if (e == hipSuccess) e = hipMalloc(&G->th, th.size() * G->elem);
  if (e == hipSuccess) e = hipMalloc(&G->v0xy, (size_t)grid->n[0] * grid->n[1] * G->elem);
  if (e == hipSuccess) e = hipMalloc(&G->lut64, 2 * m * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&G->amax_dev, 4 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&G->flag_dev, sizeof(int32_t));
  if (e == hipSuccess) e = hipHostMalloc(&G->amax_host, 4 * sizeof(double), 0);
  if (e == hipSuccess) e = hipHostMalloc(&G->flag_host, sizeof(int32_t), 0);
  if (e == hipSuccess) {
    // FP64 alphas for the reduction; the table in the step's precision.
    e = hipMemcpyAsync(G->lut64, tab.data() + 2 * m, 2 * m * sizeof(double), hipMemcpyHostToDevice, G->stream);
    if (e == hipSuccess) {
      if (G->elem == 8) {
        e = hipMemcpyAsync(G->lut, tab.data(), 4 * m * 8, hipMemcpyHostToDevice, G->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(G->coef, coef.data(), 4 * m * 8, hipMemcpyHostToDevice, G->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(G->th, th.data(), th.size() * 8, hipMemcpyHostToDevice, G->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(G->stream);
      } else {
        std::vector<float> t32(4 * m), c32(4 * m), h32(th.size());
        for (int64_t i = 0; i < 4 * m; ++i) {
          t32[i] = (float)tab[i];
          c32[i] = (float)coef[i];
        }
        for (size_t i = 0; i < th.size(); ++i) h32[i] = (float)th[i];
        e = hipMemcpyAsync(G->lut, t32.data(), 4 * m * 4, hipMemcpyHostToDevice, G->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(G->coef, c32.data(), 4 * m * 4, hipMemcpyHostToDevice, G->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(G->th, h32.data(), th.size() * 4, hipMemcpyHostToDevice, G->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(G->stream);
      }
    }
  }
  if (e != hipSuccess) {
    free_all(G);
    delete G;
    return fail(e == hipErrorOutOfMemory ? HJ_ERR_OUT_OF_MEMORY : HJ_ERR_DEVICE, "hj_grid_create: %s",
                hipGetErrorString(e));
  }
  *out = G;
  return HJ_OK;
}

hj_status hj_grid_destroy(hj_grid *G) {
  if (!G) return HJ_OK;
  (void)hipSetDevice(G->device);
  (void)hipStreamSynchronize(G->stream);
  free_all(G);
  delete G;
  return HJ_OK;
}

hj_status hj_set_target(hj_grid *G, const void *v0, int32_t dtype, int32_t where) {
  hj_status st = check_handle(G);
  if (st == HJ_OK) st = check_array(v0, dtype, where);
  if (st != HJ_OK) return st;
  if ((st = set_device(G)) != HJ_OK) return st;
  bool ok = false;
  if ((st = all_finite(G, v0, dtype, where, &ok)) != HJ_OK) return st;
  if (!ok) return fail(HJ_ERR_NONFINITE, "target contains NaN or infinity");
  if ((st = import_array(G, G->v0, v0, dtype, where)) != HJ_OK) return st;
  if ((st = reset_value(G)) != HJ_OK) return st;
  G->has_target = true;
  G->target_xy = false;
  return HJ_OK;
}

hj_status hj_set_target_cylinders(hj_grid *G, const double *cx, const double *cy, const double *r, int32_t m) {
  hj_status st = check_handle(G);
  if (st != HJ_OK) return st;
  if (!cx || !cy || !r) return fail(HJ_ERR_INVALID_ARG, "null obstacle array");
  if (m < 1) return fail(HJ_ERR_INVALID_ARG, "need at least one obstacle (m = %d)", m);
  if (bit(G->g.periodic_mask, 0) || bit(G->g.periodic_mask, 1))
    return fail(HJ_ERR_INVALID_ARG, "cylinder targets need open x and y axes");
  for (int o = 0; o < m; ++o)
    if (!isfinite(cx[o]) || !isfinite(cy[o]) || !isfinite(r[o]) || r[o] < 0)
      return fail(HJ_ERR_INVALID_ARG, "obstacle %d: need finite centre and radius >= 0", o);
  if ((st = set_device(G)) != HJ_OK) return st;
  const int K = hj::kMaxCylindersPerLaunch;
  for (int o0 = 0; o0 < m; o0 += K) {
    int cnt = m - o0 < K ? m - o0 : K;
    bool last = o0 + cnt >= m;
    if (G->elem == 4) {
      hj::CylinderArgs<float> a;
      memset(&a, 0, sizeof a);
      a.v0 = buf<float>(G->v0);
      a.v = last ? buf<float>(G->v) : nullptr;
      a.v0xy = buf<float>(G->v0xy);
      a.n0 = G->g.n[0];
      a.n1 = G->g.n[1];
      a.plane = (int64_t)G->g.n[2] * G->g.n[3];
      a.lo0 = (float)G->g.lo[0];
      a.h0 = (float)G->h[0];
      a.lo1 = (float)G->g.lo[1];
      a.h1 = (float)G->h[1];
      a.m = cnt;
      a.combine = o0 > 0;
      for (int i = 0; i < cnt; ++i) {
        a.cx[i] = (float)cx[o0 + i];
        a.cy[i] = (float)cy[o0 + i];
        a.r[i] = (float)r[o0 + i];
      }
      HJ_HIP(hj::launch_cylinders(a, S(G)));
    } else {
      hj::CylinderArgs<double> a;
      memset(&a, 0, sizeof a);
      a.v0 = buf<double>(G->v0);
      a.v = last ? buf<double>(G->v) : nullptr;
      a.v0xy = buf<double>(G->v0xy);
      a.n0 = G->g.n[0];
      a.n1 = G->g.n[1];
      a.plane = (int64_t)G->g.n[2] * G->g.n[3];
      a.lo0 = G->g.lo[0];
      a.h0 = G->h[0];
      a.lo1 = G->g.lo[1];
      a.h1 = G->h[1];
      a.m = cnt;
      a.combine = o0 > 0;
      for (int i = 0; i < cnt; ++i) {
        a.cx[i] = cx[o0 + i];
        a.cy[i] = cy[o0 + i];
        a.r[i] = r[o0 + i];
      }
      HJ_HIP(hj::launch_cylinders(a, S(G)));
    }
  }
  G->has_target = true;
  G->target_xy = true;
  return HJ_OK;
}

hj_status hj_get_cfl_dt(hj_grid *G, double *dt) {
  hj_status st = check_handle(G);
  if (st != HJ_OK) return st;
  if (!dt) return fail(HJ_ERR_INVALID_ARG, "null output");
  if ((st = set_device(G)) != HJ_OK) return st;
  if ((st = ensure_dt(G)) != HJ_OK) return st;
  *dt = G->dt_cfl;
  return HJ_OK;
}

hj_status hj_get_alpha_max(hj_grid *G, double alpha_max[4]) {
  hj_status st = check_handle(G);
  if (st != HJ_OK) return st;
  if (!alpha_max) return fail(HJ_ERR_INVALID_ARG, "null output");
  if ((st = set_device(G)) != HJ_OK) return st;
  if ((st = ensure_dt(G)) != HJ_OK) return st;
  for (int d = 0; d < 4; ++d) alpha_max[d] = G->amax[d];
  return HJ_OK;
}

hj_status hj_solve_brt(hj_grid *G, double horizon, hj_solve_info *info) {
  hj_status st = check_handle(G);
  if (st != HJ_OK) return st;
  if (!isfinite(horizon) || horizon < 0) return fail(HJ_ERR_INVALID_ARG, "horizon must be finite and >= 0");
  if (!G->has_target) return fail(HJ_ERR_NOT_READY, "no target set");
  if ((st = set_device(G)) != HJ_OK) return st;
  if ((st = ensure_dt(G)) != HJ_OK) return st;
  if (G->sch.alpha_mode != HJ_ALPHA_STATE) {
    // Algorithm 1: alpha and dt from each step's derivative range; the step
    // that would reach or pass the horizon is shortened to end on it
    if ((st = reset_value(G)) != HJ_OK) return st;
    double t = 0.0, first = 0.0, dtk = 0.0;
    int64_t n = 0, launches = 0;
    while (horizon > 0.0 && t < horizon) {
      double allowed;
      if ((st = range_alpha_update(G, &allowed)) != HJ_OK) return st;
      dtk = isinf(allowed) ? horizon - t : allowed;
      const bool last = t + dtk >= horizon;
      if (last) dtk = horizon - t;
      if ((st = step_once(G, dtk, &launches)) != HJ_OK) return st;
      if (n == 0) first = dtk;
      n += 1;
      if (last) break;
      t += dtk;
    }
    if (info) {
      info->steps = n;
      info->dt = first;
      info->dt_last = n > 0 ? dtk : 0.0;
      info->t_final = horizon;
    }
    return HJ_OK;
  }
  double dt, dt_last;
  int64_t n;
  schedule(G, horizon, &n, &dt, &dt_last);
  if ((st = reset_value(G)) != HJ_OK) return st;
  if (n > 0 && G->autotune_on && !G->autotuned && !G->launch_fixed)
    if ((st = autotune(G)) != HJ_OK) return st;
  bool timed = G->profiling && n > 0;
  hipEvent_t ev_b = nullptr, ev_e = nullptr;
  if (timed) {
    if ((st = next_events(G, &ev_b, &ev_e)) != HJ_OK) return st;
    HJ_HIP(hipEventRecord(ev_b, S(G)));
  }
  int64_t launches = 0;
  if (use_solve_graph(G, n)) {
    if ((st = solve_graph(G, n, dt, dt_last, &launches)) != HJ_OK) return st;
  } else {
    for (int64_t k = 0; k < n; ++k)
      if ((st = step_once(G, k + 1 < n ? dt : dt_last, &launches)) != HJ_OK) return st;
  }
  if (timed) {
    HJ_HIP(hipEventRecord(ev_e, S(G)));
    G->prof.solves += 1;
    G->prof.step_launches += launches;
  }
  if (info) {
    info->steps = n;
    info->dt = dt;
    info->dt_last = dt_last;
    info->t_final = horizon;
  }
  return HJ_OK;
}

hj_status hj_step(hj_grid *G, double dt, double *dt_taken) {
  hj_status st = check_handle(G);
  if (st != HJ_OK) return st;
  if (!G->has_target) return fail(HJ_ERR_NOT_READY, "no target set");
  if (isnan(dt) || isinf(dt)) return fail(HJ_ERR_INVALID_ARG, "dt must be finite");
  if ((st = set_device(G)) != HJ_OK) return st;
  if (G->sch.alpha_mode != HJ_ALPHA_STATE) {
    double allowed;
    if ((st = range_alpha_update(G, &allowed)) != HJ_OK) return st;
    if (dt <= 0) {
      if (isinf(allowed)) return fail(HJ_ERR_INVALID_ARG, "nothing moves: the CFL step is unbounded, pass dt > 0");
      dt = allowed;
    }
  } else if (dt <= 0) {
    if ((st = ensure_dt(G)) != HJ_OK) return st;
    if (isinf(G->dt_cfl)) return fail(HJ_ERR_INVALID_ARG, "nothing moves: the CFL step is unbounded, pass dt > 0");
    dt = G->dt_cfl;
  }
  int64_t launches = 0;
  if ((st = step_once(G, dt, &launches)) != HJ_OK) return st;
  if (dt_taken) *dt_taken = dt;
  return HJ_OK;
}

hj_status hj_solve_converge(hj_grid *G, double threshold, int64_t max_steps, hj_converge_info *info) {
  hj_status st = check_handle(G);
  if (st != HJ_OK) return st;
  if (isnan(threshold) || threshold < 0) return fail(HJ_ERR_INVALID_ARG, "threshold must be >= 0");
  if (max_steps < 1) return fail(HJ_ERR_INVALID_ARG, "max_steps must be >= 1");
  if (!G->has_target) return fail(HJ_ERR_NOT_READY, "no target set");
  if (G->sch.alpha_mode != HJ_ALPHA_STATE)
    return fail(HJ_ERR_UNSUPPORTED, "the convergence mode steps with the state-bound CFL step");
  if ((st = set_device(G)) != HJ_OK) return st;
  if ((st = ensure_dt(G)) != HJ_OK) return st;
  const int K = kConvergeChunk;
  if (!G->conv_acc) {
    HJ_HIP(hipMalloc((void **)&G->conv_acc, sizeof(unsigned long long)));
    HJ_HIP(hipMalloc((void **)&G->conv_state, 2 * sizeof(int32_t)));
    HJ_HIP(hipMalloc((void **)&G->conv_eps, K * sizeof(double)));
    HJ_HIP(hipHostMalloc((void **)&G->conv_host, 2 * sizeof(int32_t), 0));
    HJ_HIP(hipHostMalloc((void **)&G->conv_eps_host, K * sizeof(double), 0));
  }
  // a grid on which nothing moves takes steps of one time unit
  const double dt = isinf(G->dt_cfl) ? 1.0 : G->dt_cfl;
  if ((st = reset_value(G)) != HJ_OK) return st;
  if (G->autotune_on && !G->autotuned && !G->launch_fixed)
    if ((st = autotune(G)) != HJ_OK) return st;
  HJ_HIP(hj::launch_converge_reset(G->conv_acc, G->conv_state, S(G)));
  G->skip = G->conv_state;
  // the plane kernel folds each step's largest change into its last stage;
  // the other kernels leave it to a separate pass over V_t and V_t+1
  const bool fused = G->kernel == 2;
  G->eps_acc = fused ? G->conv_acc : nullptr;
  int64_t k = 0, steps = max_steps;
  bool stopped = false;
  double eps_last = 0.0;
  while (k < max_steps && st == HJ_OK) {
    const int64_t chunk = max_steps - k < K ? max_steps - k : K;
    int64_t launches = 0;
    for (int64_t j = 0; j < chunk && st == HJ_OK; ++j) {
      st = step_once(G, dt, &launches);  // reads v, writes w2, swaps: v new, w2 old
      if (st != HJ_OK) break;
      hipError_t e = hipSuccess;
      if (!fused)
        e = G->elem == 4 ? hj::launch_delta_max<float>(buf<const float>(G->v), buf<const float>(G->w2), G->npts,
                                                       G->conv_acc, G->skip, S(G))
                         : hj::launch_delta_max<double>(buf<const double>(G->v), buf<const double>(G->w2), G->npts,
                                                        G->conv_acc, G->skip, S(G));
      if (e == hipSuccess) e = hj::launch_converge_check(G->conv_acc, threshold, G->conv_state, G->conv_eps, (int)j, k + j, S(G));
      if (e != hipSuccess) st = fail(HJ_ERR_DEVICE, "hj_solve_converge: %s", hipGetErrorString(e));
    }
    if (st != HJ_OK) break;
    hipError_t e = hipMemcpyAsync(G->conv_host, G->conv_state, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, S(G));
    if (e == hipSuccess)
      e = hipMemcpyAsync(G->conv_eps_host, G->conv_eps, chunk * sizeof(double), hipMemcpyDeviceToHost, S(G));
    if (e == hipSuccess) e = hipStreamSynchronize(S(G));
    if (e != hipSuccess) {
      st = fail(HJ_ERR_DEVICE, "hj_solve_converge: %s", hipGetErrorString(e));
      break;
    }
    if (G->conv_host[0]) {
      steps = G->conv_host[1];
      stopped = true;
      eps_last = G->conv_eps_host[steps - 1 - k];
      // the steps after the stop did nothing, but v and w2 were swapped for
      // each of them
      if (((k + chunk - steps) & 1) != 0) {
        void *t = G->v;
        G->v = G->w2;
        G->w2 = t;
      }
      break;
    }
    eps_last = G->conv_eps_host[chunk - 1];
    k += chunk;
  }
  G->skip = nullptr;
  G->eps_acc = nullptr;
  if (st != HJ_OK) return st;
  if (info) {
    info->steps = steps;
    info->converged = stopped ? 1 : 0;
    info->reserved = 0;
    info->dt = dt;
    info->eps_last = eps_last;
  }
  return HJ_OK;
}

namespace {

// The control query of hj_optimal_control and hj_optimal_control_noalloc.
// Host arrays are staged through `staging` (7 doubles per state) when it is
// given, else through the handle's own buffer, grown as needed.
hj_status optimal_control_impl(hj_grid *G, const double *states, int64_t m, int32_t where, double *controls,
                               double *values, bool noalloc) {
  hj_status st = check_handle(G);
  if (st != HJ_OK) return st;
  if (m < 0 || (m > 0 && (!states || !controls))) return fail(HJ_ERR_INVALID_ARG, "null states or controls");
  if (where != HJ_HOST && where != HJ_DEVICE) return fail(HJ_ERR_INVALID_ARG, "unknown location %d", where);
  if (G->dyn.kind != HJ_DYN_CAR4D && G->dyn.kind != HJ_DYN_CAR4D_STEER)
    return fail(HJ_ERR_UNSUPPORTED, "the optimal control is defined for the car dynamics");
  if (noalloc && m > HJ_NOALLOC_MAX_STATES)
    return fail(HJ_ERR_INVALID_ARG, "%lld states: the no-allocation query takes at most %d", (long long)m,
                HJ_NOALLOC_MAX_STATES);
  if (m == 0) return HJ_OK;
  if ((st = set_device(G)) != HJ_OK) return st;
  const double *z = states;
  double *u = controls, *val = values;
  if (where == HJ_HOST) {
    for (int64_t i = 0; i < 4 * m; ++i)
      if (!isfinite(states[i])) return fail(HJ_ERR_INVALID_ARG, "state %lld is not finite", (long long)(i / 4));
    double *zd = nullptr;
    if (noalloc) {
      if ((st = noalloc_staging(G->device, &zd)) != HJ_OK) return st;
    } else {
      if (m > G->ctl_cap) {
        if (G->ctl_dev) HJ_HIP(hipFree(G->ctl_dev));
        G->ctl_dev = nullptr;
        G->ctl_cap = 0;
        HJ_HIP(hipMalloc((void **)&G->ctl_dev, (size_t)m * 7 * sizeof(double)));
        G->ctl_cap = m;
      }
      zd = G->ctl_dev;
    }
    HJ_HIP(hipMemcpyAsync(zd, states, m * 4 * sizeof(double), hipMemcpyHostToDevice, S(G)));
    z = zd;
    u = zd + 4 * m;
    val = values ? zd + 6 * m : nullptr;
  }
  if (G->elem == 4) {
    hj::ControlArgs<float> a;
    memset(&a, 0, sizeof a);
    a.v = buf<const float>(G->v);
    for (int d = 0; d < 4; ++d) {
      a.n[d] = G->g.n[d];
      a.lo[d] = G->g.lo[d];
      a.hi[d] = G->g.hi[d];
      a.h[d] = G->h[d];
    }
    a.periodic_mask = G->g.periodic_mask;
    a.states = z;
    a.m = m;
    a.controls = u;
    a.values = val;
    a.steer = G->dyn.kind == HJ_DYN_CAR4D_STEER;
    a.a_max = G->dyn.a_max;
    a.turn_max = a.steer ? G->dyn.steer_max : G->dyn.w_max;
    HJ_HIP(hj::launch_control(a, S(G)));
  } else {
    hj::ControlArgs<double> a;
    memset(&a, 0, sizeof a);
    a.v = buf<const double>(G->v);
    for (int d = 0; d < 4; ++d) {
      a.n[d] = G->g.n[d];
      a.lo[d] = G->g.lo[d];
      a.hi[d] = G->g.hi[d];
      a.h[d] = G->h[d];
    }
    a.periodic_mask = G->g.periodic_mask;
    a.states = z;
    a.m = m;
    a.controls = u;
    a.values = val;
    a.steer = G->dyn.kind == HJ_DYN_CAR4D_STEER;
    a.a_max = G->dyn.a_max;
    a.turn_max = a.steer ? G->dyn.steer_max : G->dyn.w_max;
    HJ_HIP(hj::launch_control(a, S(G)));
  }
  if (where == HJ_HOST) {
    HJ_HIP(hipMemcpyAsync(controls, u, m * 2 * sizeof(double), hipMemcpyDeviceToHost, S(G)));
    if (values) HJ_HIP(hipMemcpyAsync(values, val, m * sizeof(double), hipMemcpyDeviceToHost, S(G)));
    HJ_HIP(hipStreamSynchronize(S(G)));
  }
  return HJ_OK;
}

}  // namespace

hj_status hj_optimal_control(hj_grid *G, const double *states, int64_t m, int32_t where, double *controls,
                             double *values) {
  return optimal_control_impl(G, states, m, where, controls, values, false);
}

hj_status hj_optimal_control_noalloc(hj_grid *G, const double *states, int64_t m, int32_t where, double *controls,
                                     double *values) {
  return optimal_control_impl(G, states, m, where, controls, values, true);
}

hj_status hj_get_value(hj_grid *G, void *out, int32_t dtype, int32_t where) {
  hj_status st = check_handle(G);
  if (st == HJ_OK) st = check_array(out, dtype, where);
  if (st != HJ_OK) return st;
  if (!G->has_target) return fail(HJ_ERR_NOT_READY, "no target set");
  if ((st = set_device(G)) != HJ_OK) return st;
  return export_array(G, G->v, out, dtype, where);
}

hj_status hj_get_target(hj_grid *G, void *out, int32_t dtype, int32_t where) {
  hj_status st = check_handle(G);
  if (st == HJ_OK) st = check_array(out, dtype, where);
  if (st != HJ_OK) return st;
  if (!G->has_target) return fail(HJ_ERR_NOT_READY, "no target set");
  if ((st = set_device(G)) != HJ_OK) return st;
  return export_array(G, G->v0, out, dtype, where);
}

hj_status hj_set_value(hj_grid *G, const void *v, int32_t dtype, int32_t where) {
  hj_status st = check_handle(G);
  if (st == HJ_OK) st = check_array(v, dtype, where);
  if (st != HJ_OK) return st;
  if (!G->has_target) return fail(HJ_ERR_NOT_READY, "no target set");
  if ((st = set_device(G)) != HJ_OK) return st;
  bool ok = false;
  if ((st = all_finite(G, v, dtype, where, &ok)) != HJ_OK) return st;
  if (!ok) return fail(HJ_ERR_NONFINITE, "value contains NaN or infinity");
  return import_array(G, G->v, v, dtype, where);
}

hj_status hj_get_launch_info(hj_grid *G, hj_launch_info *out) {
  hj_status st = check_handle(G);
  if (st != HJ_OK) return st;
  if (!out) return fail(HJ_ERR_INVALID_ARG, "null output");
  out->kernel = G->kernel;
  out->x_chunks = G->x_chunks;
  out->target_xy = G->target_xy && G->kernel > 0;
  out->autotuned = G->autotuned;
  int vs2 = 0, ns2 = 0;
  const bool two = G->kernel == 2 && G->plane_rows == 2 && rows2_layout(G, G->plane_run, &vs2, &ns2);
  out->plane_segments = G->kernel == 2 ? (two ? ns2 : (G->plane_run == 3 ? 1 : G->n_seg)) : 0;
  out->theta_run = G->kernel == 2 ? G->plane_run : hj::run_length((int)G->elem, G->g.n[3]);
  out->span_blocks = G->kernel == 2 && !two && (G->plane_run == 3 || G->n_seg == 1) ? G->span_blocks : 0;
  out->plane_rows = G->kernel == 2 ? (two ? 2 : 1) : 0;
  out->reserved = 0;
  out->solve_graph = G->sch.alpha_mode == HJ_ALPHA_STATE && use_solve_graph(G, 2) ? 1 : 0;
  // arrays per stage: read the stencil input, write the output; stage 2 of
  // TVD-RK2 also reads V^n; the clamp reads V0 unless it is the xy table
  double arrays;
  bool v0full = G->sch.clamp == HJ_CLAMP_MIN_V0 && !out->target_xy;
  if (G->sch.integrator == HJ_EULER)
    arrays = 2 + (v0full ? 1 : 0);
  else
    arrays = 2 + 3 + (v0full ? 1 : 0);
  out->bytes_per_point_step = arrays * (double)G->elem;
  return HJ_OK;
}

hj_status hj_autotune(hj_grid *G) {
  hj_status st = check_handle(G);
  if (st != HJ_OK) return st;
  if (!G->has_target) return fail(HJ_ERR_NOT_READY, "no target set");
  if ((st = set_device(G)) != HJ_OK) return st;
  if (G->launch_fixed) return HJ_OK;
  G->autotuned = false;
  return autotune(G);
}

hj_status hj_set_autotune(hj_grid *G, int32_t enable) {
  hj_status st = check_handle(G);
  if (st != HJ_OK) return st;
  G->autotune_on = enable != 0;
  return HJ_OK;
}

hj_status hj_get_num_points(hj_grid *G, int64_t *n) {
  hj_status st = check_handle(G);
  if (st != HJ_OK) return st;
  if (!n) return fail(HJ_ERR_INVALID_ARG, "null output");
  *n = G->npts;
  return HJ_OK;
}

hj_status hj_set_profiling(hj_grid *G, int32_t enable) {
  hj_status st = check_handle(G);
  if (st != HJ_OK) return st;
  if ((st = set_device(G)) != HJ_OK) return st;
  if ((st = fold_events(G)) != HJ_OK) return st;
  G->profiling = enable != 0;
  G->prof = {0, 0, 0.0};
  return HJ_OK;
}

hj_status hj_get_profile(hj_grid *G, hj_profile *out) {
  hj_status st = check_handle(G);
  if (st != HJ_OK) return st;
  if (!out) return fail(HJ_ERR_INVALID_ARG, "null output");
  if ((st = set_device(G)) != HJ_OK) return st;
  if ((st = fold_events(G)) != HJ_OK) return st;
  *out = G->prof;
  return HJ_OK;
}

}  // extern "C"

// ===========================================================================
// Batched solves
// ===========================================================================

// Streams of the concurrent batch mode: one per hardware queue a process
// gets by default, so that independent solves can run side by side.
constexpr int kBatchLanes = 4;

struct hj_batch {
  std::vector<hj_grid *> g;
  int m = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;  // private stream the graph is captured on
  int device = 0;
  size_t elem = 4;
  int deriv = 0;
  bool rk2 = false, sg = false, ball = false;
  int32_t x_planes = 0;  // 0: automatic
  bool plane_allowed = true;  // launch and graph modes may run the batched plane kernel (HJ_BATCH_KERNEL)
  int64_t spin_limit = (int64_t)1 << 21;
  int cus = 0;

  void *inst_dev = nullptr;   // BatchInst<T>[m], sorted by step count
  void *inst_host = nullptr;  // pinned staging of the same
  int32_t *ints_dev = nullptr;   // tile_end[m] | start[nphase + 1] | active[nphase]
  int32_t *ints_host = nullptr;  // pinned
  size_t ints_cap = 0;           // entries
  hipEvent_t staged = nullptr;   // the last upload from the pinned buffers
  hj::BatchQueue *queue = nullptr;
  int32_t *err_host = nullptr;   // pinned

  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<int64_t> gkey;
  int32_t graph_nodes = 0;

  // HJ_BATCH_STREAMS: private lanes (created on first use), the fork event
  // they wait on and the join events the batch stream waits on
  hipStream_t lanes[kBatchLanes] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kBatchLanes] = {};

  hj_batch_info info = {};
};

namespace {

void batch_free(hj_batch *b) {
  for (int k = 0; k < kBatchLanes; ++k) {
    if (b->lanes[k]) (void)hipStreamDestroy(b->lanes[k]);
    if (b->join[k]) (void)hipEventDestroy(b->join[k]);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->staged) (void)hipEventDestroy(b->staged);
  void *dev[] = {b->inst_dev, b->ints_dev, b->queue};
  for (void *p : dev)
    if (p) (void)hipFree(p);
  void *host[] = {b->inst_host, b->ints_host, b->err_host};
  for (void *p : host)
    if (p) (void)hipHostFree(p);
}

constexpr int32_t kBatchDefaultXPlanes = 16;
constexpr int32_t kBatchPlaneDefaultXPlanes = 32;  // the batched plane kernel's x planes per block
constexpr int64_t kServerBlocks = 1024;
constexpr int64_t kServerAlonePoints = (int64_t)4 << 20;  // grids this large step on their own kernel
constexpr int64_t kServerFillPoints = kServerAlonePoints;  // small-first: nodes that fill the device
constexpr double kServerAgeMs = 5.0;  // small-first: the default age after which a request goes first

double host_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int32_t batch_x_planes(const hj_batch *b, bool plane = false) {
  return b->x_planes > 0 ? b->x_planes : (plane ? kBatchPlaneDefaultXPlanes : kBatchDefaultXPlanes);
}

// x chunks of a grid in a batch: ceil(N_x / x planes per tile)
int batch_chunks(const hj_batch *b, const hj_grid *G) {
  int xp = batch_x_planes(b);
  return (G->g.n[0] + xp - 1) / xp;
}

// The batched plane kernel's description of instance G, x_planes x planes
// per block: the handle's plane run length and v split (runs of 3 with more
// runs than that kernel's blocks hold take the handle's other run length),
// or false where its planes fit no batched plane block.
template <typename T>
bool batch_plane_args(hj_grid *G, int32_t x_planes, hj::StreamArgs<T> *out, int *threads, size_t *lds) {
  if (!G->plane_ok) return false;
  const int runs[2] = {G->plane_run, G->plane_run_alt};
  for (int r : runs) {
    if (r == 0) continue;
    hj::StreamArgs<T> a = stream_args<T>(G, true, r);
    a.skip = nullptr;
    a.span = 0;
    const int nx = G->g.n[0];
    a.chunk_len = x_planes < nx ? x_planes : nx;
    a.n_chunks = (nx + a.chunk_len - 1) / a.chunk_len;
    if (hj::plane_multi_fits<T>(a, threads, lds)) {
      *out = a;
      return true;
    }
  }
  return false;
}

template <typename T>
hj::StreamArgs<T> batch_stream_args(hj_grid *G, int n_chunks) {
  hj::StreamArgs<T> a = stream_args<T>(G, false);
  a.skip = nullptr;
  a.blocks_per_chunk = (a.slab_runs + hj::kStreamBlock - 1) / hj::kStreamBlock;
  int nx = G->g.n[0];
  if (n_chunks > nx) n_chunks = nx;
  a.chunk_len = (nx + n_chunks - 1) / n_chunks;
  a.n_chunks = (nx + a.chunk_len - 1) / a.chunk_len;
  return a;
}

struct BatchPlan {
  std::vector<int> order;      // sorted position -> instance
  std::vector<int64_t> steps;  // per instance
  std::vector<double> dt, dt_last;
  std::vector<int32_t> tiles;  // per sorted position
  std::vector<int32_t> tile_end, start, active;
  int nphase = 0, pps = 1;
  // launch classes: class c holds sorted positions cls_begin[c] ..
  // cls_begin[c+1]-1 (tile_end restarts at each class) and runs the batched
  // plane kernel (cls_plane[c]) or the streaming tiles; work-items and LDS
  // bytes per plane block over the class's positions up to i
  bool plane = false;  // some class runs the plane kernel
  std::vector<int> cls_begin;
  std::vector<uint8_t> cls_plane;
  std::vector<int32_t> threads;
  std::vector<int64_t> lds;
};

// Launch classes of the batched plane kernel, by the waves of an instance's
// blocks: 1-2, 3-4 and 5-12; the instances it does not take (among them
// those with runs of one theta node) form the streaming class.  A workgroup is dispatched only where all its waves'
// registers fit, so a block sized for a larger instance would hold a small
// instance's CU share idle; each class runs its own launches, on its own
// lane beside the others.
constexpr int kStreamClass = 3;
int plane_class(int threads) {
  const int w = (threads + 63) / 64;
  return w <= 2 ? 0 : (w <= 4 ? 1 : 2);
}
static_assert(kStreamClass + 1 <= kBatchLanes, "a lane per class");

// Step schedules, the sorted order and the host tables of one batch solve
// (plane_mode: the launches may run the batched plane kernel, which they do
// when it takes every instance).
template <typename T>
hj_status batch_plan(hj_batch *b, const double *horizons, BatchPlan *P, bool plane_mode) {
  hj_status st;
  const int m = b->m;
  P->steps.resize(m);
  P->dt.resize(m);
  P->dt_last.resize(m);
  int64_t points = 0;
  for (int j = 0; j < m; ++j) {
    hj_grid *G = b->g[j];
    if ((st = ensure_dt(G)) != HJ_OK) return st;
    schedule(G, horizons[j], &P->steps[j], &P->dt[j], &P->dt_last[j]);
    if (P->steps[j] > ((int64_t)1 << 24)) return fail(HJ_ERR_INVALID_ARG, "instance %d: %lld steps", j, (long long)P->steps[j]);
    points += G->npts;
  }
  // the batched plane kernel's description of the instances it takes
  const bool try_plane = plane_mode && b->plane_allowed;
  std::vector<hj::StreamArgs<T>> pa(try_plane ? m : 0);
  std::vector<int> thr(m, 0), cls(m, kStreamClass);
  std::vector<size_t> bytes(m, 0);
  for (int j = 0; j < m && try_plane; ++j)
    if (batch_plane_args<T>(b->g[j], batch_x_planes(b, true), &pa[j], &thr[j], &bytes[j]))
      cls[j] = plane_class(thr[j]);
  P->order.resize(m);
  for (int j = 0; j < m; ++j) P->order[j] = j;
  std::stable_sort(P->order.begin(), P->order.end(), [&](int x, int y) {
    return cls[x] != cls[y] ? cls[x] < cls[y] : P->steps[x] > P->steps[y];
  });
  P->cls_begin.assign(1, 0);
  P->cls_plane.assign(1, cls[P->order[0]] != kStreamClass);
  for (int i = 1; i < m; ++i)
    if (cls[P->order[i]] != cls[P->order[i - 1]]) {
      P->cls_begin.push_back(i);
      P->cls_plane.push_back(cls[P->order[i]] != kStreamClass);
    }
  P->cls_begin.push_back(m);
  P->plane = std::find(P->cls_plane.begin(), P->cls_plane.end(), 1) != P->cls_plane.end();
  b->info.classes = (int32_t)P->cls_plane.size();
  P->pps = b->rk2 ? 2 : 1;
  int64_t maxn = 0;
  for (int j = 0; j < m; ++j) maxn = std::max(maxn, P->steps[j]);
  P->nphase = (int)(maxn * P->pps);
  hj::BatchInst<T> *inst = static_cast<hj::BatchInst<T> *>(b->inst_host);
  P->tiles.resize(m);
  P->tile_end.resize(m);
  P->threads.assign(m, 0);
  P->lds.assign(m, 0);
  b->info.plane_kernel = P->plane ? 1 : 0;
  int64_t acc = 0;
  for (int i = 0; i < m; ++i) {
    const int j = P->order[i];
    hj_grid *G = b->g[j];
    hj::BatchInst<T> &in = inst[i];
    memset(&in, 0, sizeof in);
    const bool first = std::find(P->cls_begin.begin(), P->cls_begin.end(), i) != P->cls_begin.end();
    if (first) acc = 0;  // each class's tile prefix starts at 0
    if (cls[j] != kStreamClass) {
      in.a = pa[j];
      P->threads[i] = std::max(thr[j], first ? 0 : P->threads[i - 1]);
      P->lds[i] = std::max((int64_t)bytes[j], first ? (int64_t)0 : P->lds[i - 1]);
    } else {
      in.a = batch_stream_args<T>(G, batch_chunks(b, G));
    }
    in.v0 = buf<const T>(G->v0);
    in.va = buf<T>(G->v);
    in.vb = buf<T>(G->w2);
    in.w1 = b->rk2 ? buf<T>(G->w1) : nullptr;
    in.dt = (T)P->dt[j];
    in.dt_last = (T)P->dt_last[j];
    in.steps = (int32_t)P->steps[j];
    in.rk2 = b->rk2 ? 1 : 0;
    in.clamp = G->sch.clamp == HJ_CLAMP_MIN_V0 ? 1 : 0;
    const int64_t tiles = (int64_t)in.a.blocks_per_chunk * in.a.n_chunks;
    if (tiles >= ((int64_t)1 << 30)) return fail(HJ_ERR_UNSUPPORTED, "batch too large");
    in.tiles = (int32_t)tiles;
    P->tiles[i] = in.tiles;
    acc += in.tiles;
    if (acc >= ((int64_t)1 << 30)) return fail(HJ_ERR_UNSUPPORTED, "batch too large");
    P->tile_end[i] = (int32_t)acc;
  }
  // active[p]: instances of the first class still running in phase p (the
  // one class of the streaming tiles and the persistent kernel's work list)
  P->active.resize(P->nphase);
  P->start.resize(P->nphase + 1);
  int64_t items = 0, sweep = 0;
  for (size_t c = 0; c + 1 < P->cls_begin.size(); ++c) {
    const int c0 = P->cls_begin[c];
    int act = P->cls_begin[c + 1] - c0;
    sweep += P->tile_end[c0 + act - 1];
    for (int p = 0; p < P->nphase; ++p) {
      int64_t k = p / P->pps;
      while (act > 0 && P->steps[P->order[c0 + act - 1]] <= k) --act;
      if (c == 0) {
        P->active[p] = act;
        P->start[p] = (int32_t)items;
      }
      if (act > 0) items += P->tile_end[c0 + act - 1];
      if (items >= ((int64_t)1 << 31) - 1) return fail(HJ_ERR_UNSUPPORTED, "batch work list too long");
    }
  }
  P->start[P->nphase] = (int32_t)items;
  b->info.tiles_per_sweep = sweep;
  b->info.work_items = items;
  b->info.points = points;
  return HJ_OK;
}

// Upload the instance table and the int tables (tile_end | start | active)
// from the pinned staging buffers (which must not be rewritten before the
// copy has run: the caller waits on b->staged first).
template <typename T>
hj_status batch_upload(hj_batch *b, const BatchPlan &P) {
  size_t need = (size_t)b->m + P.start.size() + P.active.size();
  if (need > b->ints_cap) {
    HJ_HIP(hipStreamSynchronize(b->stream));  // earlier launches may still read the old tables
    if (b->ints_dev) HJ_HIP(hipFree(b->ints_dev));
    if (b->ints_host) HJ_HIP(hipHostFree(b->ints_host));
    b->ints_dev = nullptr;
    b->ints_host = nullptr;
    b->ints_cap = 0;
    HJ_HIP(hipMalloc(&b->ints_dev, need * sizeof(int32_t)));
    HJ_HIP(hipHostMalloc(&b->ints_host, need * sizeof(int32_t), 0));
    b->ints_cap = need;
  }
  int32_t *h = b->ints_host;
  memcpy(h, P.tile_end.data(), b->m * sizeof(int32_t));
  memcpy(h + b->m, P.start.data(), P.start.size() * sizeof(int32_t));
  memcpy(h + b->m + P.start.size(), P.active.data(), P.active.size() * sizeof(int32_t));
  HJ_HIP(hipMemcpyAsync(b->ints_dev, h, need * sizeof(int32_t), hipMemcpyHostToDevice, b->stream));
  HJ_HIP(hipMemcpyAsync(b->inst_dev, b->inst_host, b->m * sizeof(hj::BatchInst<T>), hipMemcpyHostToDevice,
                        b->stream));
  HJ_HIP(hipEventRecord(b->staged, b->stream));
  return HJ_OK;
}

hj_status batch_lanes(hj_batch *b) {
  for (int k = 0; k < kBatchLanes; ++k) {
    if (!b->lanes[k]) HJ_HIP(hipStreamCreateWithFlags(&b->lanes[k], hipStreamNonBlocking));
    if (!b->join[k]) HJ_HIP(hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming));
  }
  if (!b->fork) HJ_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
  return HJ_OK;
}

// The launches of class c on stream s: one per (step, stage) over the
// class's instances still running.
template <typename T>
hj_status batch_enqueue_class(hj_batch *b, const BatchPlan &P, int c, hipStream_t s, int32_t *nodes) {
  const int c0 = P.cls_begin[c], c1 = P.cls_begin[c + 1];
  const hj::BatchInst<T> *inst = static_cast<const hj::BatchInst<T> *>(b->inst_dev) + c0;
  const int32_t *tile_end = b->ints_dev + c0;
  int act = c1 - c0;
  for (int p = 0; p < P.nphase; ++p) {
    const int64_t k = p / P.pps;
    while (act > 0 && P.steps[P.order[c0 + act - 1]] <= k) --act;
    if (act == 0) break;
    const int last = c0 + act - 1;
    if (P.cls_plane[c])
      HJ_HIP(hj::launch_plane_multi<T>(inst, tile_end, act, P.tile_end[last], P.threads[last], (size_t)P.lds[last],
                                       (int)k, p % P.pps, b->deriv, b->sg, b->ball, s));
    else
      HJ_HIP(hj::launch_multi<T>(inst, tile_end, act, P.tile_end[last], (int)k, p % P.pps, b->deriv, b->sg, b->ball,
                                 s));
    *nodes += 1;
  }
  return HJ_OK;
}

// One launch per (step, stage) and class, each over the class's instances
// still running; with several classes, class c runs on lane c, forked from
// s and joined back into it (also while s is being captured into a graph).
template <typename T>
hj_status batch_enqueue_launches(hj_batch *b, const BatchPlan &P, hipStream_t s, int32_t *nodes) {
  *nodes = 0;
  const int ncls = (int)P.cls_begin.size() - 1;
  if (ncls == 1) return batch_enqueue_class<T>(b, P, 0, s, nodes);
  hj_status st;
  if ((st = batch_lanes(b)) != HJ_OK) return st;
  HJ_HIP(hipEventRecord(b->fork, s));
  for (int c = 0; c < ncls; ++c) HJ_HIP(hipStreamWaitEvent(b->lanes[c], b->fork, 0));
  st = HJ_OK;
  for (int c = 0; c < ncls && st == HJ_OK; ++c)
    st = batch_enqueue_class<T>(b, P, c, b->lanes[c], nodes);
  // join every forked lane, also after a failed launch
  for (int c = 0; c < ncls; ++c) {
    HJ_HIP(hipEventRecord(b->join[c], b->lanes[c]));
    HJ_HIP(hipStreamWaitEvent(s, b->join[c], 0));
  }
  return st;
}

template <typename T>
hj_status batch_solve_t(hj_batch *b, const double *horizons, int32_t mode, hj_solve_info *infos) {
  hj_status st;
  HJ_HIP(hipEventSynchronize(b->staged));  // the pinned tables are free again
  BatchPlan P;
  if ((st = batch_plan<T>(b, horizons, &P, mode != HJ_BATCH_PERSISTENT)) != HJ_OK) return st;
  if (P.nphase > 0) {
    if ((st = batch_upload<T>(b, P)) != HJ_OK) return st;
    if (mode == HJ_BATCH_LAUNCHES) {
      int32_t nodes;
      if ((st = batch_enqueue_launches<T>(b, P, b->stream, &nodes)) != HJ_OK) return st;
    } else if (mode == HJ_BATCH_GRAPH) {
      std::vector<int64_t> key;
      key.push_back(P.pps);
      key.push_back(P.plane ? 1 : 0);
      for (int c : P.cls_begin) key.push_back(c);
      for (uint8_t c : P.cls_plane) key.push_back(c);
      for (int i = 0; i < b->m; ++i) {
        key.push_back(P.steps[P.order[i]]);
        key.push_back(P.tiles[i]);
        key.push_back(P.threads[i]);
        key.push_back(P.lds[i]);
      }
      if (!b->gexec || key != b->gkey) {
        if (b->gexec) HJ_HIP(hipGraphExecDestroy(b->gexec));
        if (b->graph) HJ_HIP(hipGraphDestroy(b->graph));
        b->gexec = nullptr;
        b->graph = nullptr;
        b->gkey.clear();
        HJ_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        int32_t nodes = 0;
        st = batch_enqueue_launches<T>(b, P, b->cap, &nodes);
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamEndCapture(b->cap, &gr);
        if (st != HJ_OK) {
          if (gr) (void)hipGraphDestroy(gr);
          return st;
        }
        HJ_HIP(e);
        b->graph = gr;
        HJ_HIP(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
        b->gkey = key;
        b->graph_nodes = nodes;
      }
      HJ_HIP(hipGraphLaunch(b->gexec, b->stream));
    } else {
      hj::PersistArgs<T> pa;
      pa.inst = static_cast<const hj::BatchInst<T> *>(b->inst_dev);
      pa.tile_end = b->ints_dev;
      pa.start = b->ints_dev + b->m;
      pa.active = b->ints_dev + b->m + P.start.size();
      pa.queue = b->queue;
      pa.nphase = P.nphase;
      pa.phases_per_step = P.pps;
      pa.spin_limit = b->spin_limit;
      int per_cu = hj::persistent_blocks_per_cu<T>(b->deriv, b->sg, b->ball);
      int64_t blocks = (int64_t)per_cu * b->cus;
      if (blocks > b->info.work_items) blocks = b->info.work_items;
      if (blocks < 1) blocks = 1;
      b->info.persistent_blocks = (int32_t)blocks;
      HJ_HIP(hj::launch_batch_reset(b->queue, b->m, b->stream));
      HJ_HIP(hj::launch_persistent<T>(pa, (int)blocks, b->deriv, b->sg, b->ball, b->stream));
      HJ_HIP(hipMemcpyAsync(b->err_host, &b->queue->error, sizeof(int32_t), hipMemcpyDeviceToHost, b->stream));
      HJ_HIP(hipStreamSynchronize(b->stream));
      if (*b->err_host != 0)
        return fail(HJ_ERR_DEVICE,
                    "persistent batch: a tile waited longer than the spin limit for its previous phase; the "
                    "instances' values are undefined");
    }
  }
  // each instance's result is V^n: V0 (n = 0), vb (n odd: now becomes v) or va
  for (int j = 0; j < b->m; ++j) {
    hj_grid *G = b->g[j];
    int64_t n = P.steps[j];
    if (n == 0) {
      HJ_HIP(hj::launch_copy<T>(buf<T>(G->v), buf<const T>(G->v0), G->npts, b->stream));
    } else if (n & 1) {
      void *t = G->v;
      G->v = G->w2;
      G->w2 = t;
    }
    if (infos) {
      infos[j].steps = n;
      infos[j].dt = P.dt[j];
      infos[j].dt_last = P.dt_last[j];
      infos[j].t_final = horizons[j];
    }
  }
  b->info.graph_nodes = b->graph_nodes;
  return HJ_OK;
}

hj_status check_batch(hj_batch *b) {
  if (!b) return fail(HJ_ERR_INVALID_ARG, "null batch");
  return HJ_OK;
}

// HJ_BATCH_STREAMS: each instance runs its own single-grid solve (its own
// kernel and launch configuration, its own solve graph) on one of the
// batch's lanes, so that small solves share the device.  The lanes fork from
// the batch stream and the batch stream joins them at the end; instances go
// to the least-loaded lane in decreasing order of work (nodes x steps).
hj_status batch_solve_streams(hj_batch *b, const double *horizons, hj_solve_info *infos) {
  hj_status st;
  if ((st = batch_lanes(b)) != HJ_OK) return st;
  std::vector<std::pair<double, int>> work((size_t)b->m);
  b->info.points = 0;
  b->info.work_items = 0;  // no tiles: every instance runs its own solve
  for (int j = 0; j < b->m; ++j) {
    hj_grid *G = b->g[j];
    b->info.points += G->npts;
    if ((st = ensure_dt(G)) != HJ_OK) return st;
    double dt, dt_last;
    int64_t n;
    schedule(G, horizons[j], &n, &dt, &dt_last);
    work[(size_t)j] = {-(double)G->npts * (double)n, j};
  }
  std::stable_sort(work.begin(), work.end());
  HJ_HIP(hipEventRecord(b->fork, b->stream));
  for (int k = 0; k < kBatchLanes; ++k) HJ_HIP(hipStreamWaitEvent(b->lanes[k], b->fork, 0));
  double load[kBatchLanes] = {};
  st = HJ_OK;
  for (const auto &w : work) {
    int k = 0;
    for (int i = 1; i < kBatchLanes; ++i)
      if (load[i] < load[k]) k = i;
    load[k] -= w.first;
    hj_grid *G = b->g[(size_t)w.second];
    hipStream_t own = G->stream;
    G->stream = b->lanes[k];
    st = hj_solve_brt(G, horizons[w.second], infos ? &infos[w.second] : nullptr);
    G->stream = own;
    if (st != HJ_OK) break;
  }
  // join every lane, also after a failed solve, so that the batch stream is
  // ordered after whatever was enqueued
  for (int k = 0; k < kBatchLanes; ++k) {
    HJ_HIP(hipEventRecord(b->join[k], b->lanes[k]));
    HJ_HIP(hipStreamWaitEvent(b->stream, b->join[k], 0));
  }
  return st;
}

hj_status check_horizons(const hj_batch *b, const double *horizons) {
  if (!horizons) return fail(HJ_ERR_INVALID_ARG, "null horizons");
  for (int j = 0; j < b->m; ++j)
    if (!isfinite(horizons[j]) || horizons[j] < 0)
      return fail(HJ_ERR_INVALID_ARG, "horizon %d must be finite and >= 0", j);
  for (int j = 0; j < b->m; ++j)
    if (!b->g[j]->has_target) return fail(HJ_ERR_NOT_READY, "instance %d has no target", j);
  return HJ_OK;
}

}  // namespace

extern "C" {

hj_status hj_batch_create(hj_grid *const *grids, int32_t m, hj_batch **out) {
  if (!out) return fail(HJ_ERR_INVALID_ARG, "null output handle pointer");
  *out = nullptr;
  if (!grids || m < 1 || m > hj::kMaxBatch)
    return fail(HJ_ERR_INVALID_ARG, "need 1..%d grid handles (got %d)", hj::kMaxBatch, m);
  hj_grid *G0 = grids[0];
  for (int j = 0; j < m; ++j) {
    hj_grid *G = grids[j];
    if (!G) return fail(HJ_ERR_INVALID_ARG, "grid %d is null", j);
    for (int i = 0; i < j; ++i)
      if (grids[i] == G) return fail(HJ_ERR_INVALID_ARG, "grid %d appears twice", j);
    if (G->elem != G0->elem || G->sch.deriv != G0->sch.deriv || G->sch.integrator != G0->sch.integrator)
      return fail(HJ_ERR_UNSUPPORTED, "grid %d: a batch needs one precision, derivative and integrator", j);
    if (G->device != G0->device || G->stream != G0->stream)
      return fail(HJ_ERR_UNSUPPORTED, "grid %d: a batch needs one device and one stream", j);
    if (!G->stream_ok)
      return fail(HJ_ERR_UNSUPPORTED, "grid %d: batched solves need a periodic theta axis and < 4 GiB arrays", j);
    if (G->sch.alpha_mode != HJ_ALPHA_STATE)
      return fail(HJ_ERR_UNSUPPORTED, "grid %d: batched solves need the state-bound alpha", j);
  }
  hj_batch *b = new (std::nothrow) hj_batch;
  if (!b) return fail(HJ_ERR_OUT_OF_MEMORY, "host allocation failed");
  b->g.assign(grids, grids + m);
  b->m = m;
  b->stream = G0->stream;
  b->device = G0->device;
  b->elem = G0->elem;
  b->deriv = G0->sch.deriv;
  b->rk2 = G0->sch.integrator == HJ_TVD_RK2;
  for (hj_grid *G : b->g) {
    if (G->sig[0] != 0.0 || G->sig[1] != 0.0) b->sg = true;
    if (G->ball_mask != 0) b->ball = true;
  }
  hipError_t e = hipSetDevice(b->device);
  size_t inst_bytes = (size_t)m * (b->elem == 4 ? sizeof(hj::BatchInst<float>) : sizeof(hj::BatchInst<double>));
  if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc(&b->inst_dev, inst_bytes);
  if (e == hipSuccess) e = hipHostMalloc(&b->inst_host, inst_bytes, 0);
  if (e == hipSuccess) e = hipMalloc((void **)&b->queue, sizeof(hj::BatchQueue));
  if (e == hipSuccess) e = hipHostMalloc((void **)&b->err_host, sizeof(int32_t), 0);
  if (e == hipSuccess) e = hipEventRecord(b->staged, b->stream);
  if (e != hipSuccess) {
    batch_free(b);
    delete b;
    return fail(e == hipErrorOutOfMemory ? HJ_ERR_OUT_OF_MEMORY : HJ_ERR_DEVICE, "hj_batch_create: %s",
                hipGetErrorString(e));
  }
  b->info.m = m;
  const char *kern = getenv("HJ_BATCH_KERNEL");
  b->plane_allowed = !(kern && !strcmp(kern, "stream"));
  *out = b;
  return HJ_OK;
}

hj_status hj_batch_destroy(hj_batch *b) {
  if (!b) return HJ_OK;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  batch_free(b);
  delete b;
  return HJ_OK;
}

hj_status hj_batch_solve(hj_batch *b, const double *horizons, int32_t mode, hj_solve_info *infos) {
  hj_status st = check_batch(b);
  if (st != HJ_OK) return st;
  if (mode != HJ_BATCH_LAUNCHES && mode != HJ_BATCH_GRAPH && mode != HJ_BATCH_PERSISTENT && mode != HJ_BATCH_STREAMS)
    return fail(HJ_ERR_INVALID_ARG, "unknown batch mode %d", mode);
  if ((st = check_horizons(b, horizons)) != HJ_OK) return st;
  HJ_HIP(hipSetDevice(b->device));
  if (mode == HJ_BATCH_STREAMS) return batch_solve_streams(b, horizons, infos);
  return b->elem == 4 ? batch_solve_t<float>(b, horizons, mode, infos) : batch_solve_t<double>(b, horizons, mode, infos);
}

hj_status hj_batch_set_tile(hj_batch *b, int32_t x_planes) {
  hj_status st = check_batch(b);
  if (st != HJ_OK) return st;
  if (x_planes < 0) return fail(HJ_ERR_INVALID_ARG, "x_planes must be >= 0");
  b->x_planes = x_planes;
  return HJ_OK;
}

hj_status hj_batch_set_spin_limit(hj_batch *b, int64_t polls) {
  hj_status st = check_batch(b);
  if (st != HJ_OK) return st;
  if (polls < 0) return fail(HJ_ERR_INVALID_ARG, "spin limit must be >= 0");
  b->spin_limit = polls;
  return HJ_OK;
}

hj_status hj_batch_autotune(hj_batch *b, const double *horizons, int32_t mode, int32_t *x_planes_out) {
  hj_status st = check_batch(b);
  if (st != HJ_OK) return st;
  if (mode != HJ_BATCH_LAUNCHES && mode != HJ_BATCH_GRAPH && mode != HJ_BATCH_PERSISTENT)
    return fail(HJ_ERR_INVALID_ARG, "batch mode %d has no tile length to tune", mode);
  if ((st = check_horizons(b, horizons)) != HJ_OK) return st;
  HJ_HIP(hipSetDevice(b->device));
  const int32_t cand[] = {4, 8, 12, 16, 24, 32, 48, 80};
  hipEvent_t e0, e1;
  HJ_HIP(hipEventCreate(&e0));
  HJ_HIP(hipEventCreate(&e1));
  int32_t keep = b->x_planes, best_t = 0;
  float best = INFINITY;
  for (int32_t t : cand) {
    b->x_planes = t;
    for (int rep = 0; rep < 2 && st == HJ_OK; ++rep) {  // the first run may capture a graph
      if ((st = hipEventRecord(e0, b->stream) == hipSuccess ? HJ_OK : HJ_ERR_DEVICE) != HJ_OK) break;
      st = b->elem == 4 ? batch_solve_t<float>(b, horizons, mode, nullptr) : batch_solve_t<double>(b, horizons, mode, nullptr);
      if (st != HJ_OK) break;
      if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) st = HJ_ERR_DEVICE;
    }
    if (st != HJ_OK) break;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) {
      best = ms;
      best_t = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != HJ_OK) {
    b->x_planes = keep;
    return st == HJ_ERR_DEVICE ? fail(HJ_ERR_DEVICE, "hj_batch_autotune: device error") : st;
  }
  b->x_planes = best_t;
  if (x_planes_out) *x_planes_out = best_t;
  return HJ_OK;
}

hj_status hj_batch_get_info(hj_batch *b, hj_batch_info *out) {
  hj_status st = check_batch(b);
  if (st != HJ_OK) return st;
  if (!out) return fail(HJ_ERR_INVALID_ARG, "null output");
  b->info.x_planes = batch_x_planes(b, b->info.plane_kernel != 0);
  *out = b->info;
  return HJ_OK;
}

}  // extern "C"

// ===========================================================================
// Serving: continuous batching of re-solves
// ===========================================================================

struct hj_server {
  hj_server_desc d;
  hipStream_t stream = nullptr;
  int device = 0;
  size_t elem = 4;

  struct Slot {
    hj_grid *g = nullptr;
    int64_t bytes = 0;
    bool busy = false;
    int64_t last_use = 0;
  };
  std::vector<Slot> slots;
  int64_t slot_bytes = 0;

  struct Req {
    hj_grid_desc g;
    hj_dynamics_desc dyn;
    std::vector<double> cx, cy, r;
    double horizon = 0;
    int state = 0;  // 0 queued, 1 running, 2 finishing (event pending), 3 complete
    int slot = -1;
    int64_t n = 0, k = 0;
    double dt = 0, dt_last = 0;
    double submitted_s = 0;  // host clock at submission (seconds)
    hipEvent_t ev = nullptr;
  };
  std::map<int64_t, Req> reqs;
  std::deque<int64_t> queue;
  std::vector<int64_t> running;
  int64_t next_id = 1;

  static const int kRing = 2;  // device tables (ticks) in flight: bounds how far the host runs ahead
  void *inst_host[kRing] = {}, *inst_dev[kRing] = {};
  int32_t *tile_host[kRing] = {}, *tile_dev[kRing] = {};
  hipEvent_t ring_ev[kRing] = {};
  int ring = 0;
  std::vector<hipEvent_t> ev_free;

  hj_server_stats stats = {};
};

namespace {

void server_free(hj_server *S) {
  for (auto &kv : S->reqs)
    if (kv.second.ev) (void)hipEventDestroy(kv.second.ev);
  for (hipEvent_t e : S->ev_free) (void)hipEventDestroy(e);
  for (auto &sl : S->slots)
    if (sl.g) (void)hj_grid_destroy(sl.g);
  for (int i = 0; i < hj_server::kRing; ++i) {
    if (S->ring_ev[i]) (void)hipEventDestroy(S->ring_ev[i]);
    if (S->inst_dev[i]) (void)hipFree(S->inst_dev[i]);
    if (S->tile_dev[i]) (void)hipFree(S->tile_dev[i]);
    if (S->inst_host[i]) (void)hipHostFree(S->inst_host[i]);
    if (S->tile_host[i]) (void)hipHostFree(S->tile_host[i]);
  }
}

bool same_problem(const hj_grid *G, const hj_grid_desc &g, const hj_dynamics_desc &dyn) {
  return memcmp(&G->g, &g, sizeof g) == 0 && memcmp(&G->dyn, &dyn, sizeof dyn) == 0;
}

// Device bytes a slot of this grid holds (the handle's arrays).
int64_t slot_bytes_of(const hj_server *S, const hj_grid_desc &g) {
  int64_t n = (int64_t)g.n[0] * g.n[1] * g.n[2] * g.n[3];
  int arrays = S->d.scheme.integrator == HJ_TVD_RK2 ? 4 : 3;
  int64_t m = (int64_t)g.n[2] * g.n[3];
  return (int64_t)S->elem * (arrays * n + 8 * m + (int64_t)g.n[0] * g.n[1]) + 16 * m;
}

hj_status server_event(hj_server *S, hipEvent_t *e) {
  if (!S->ev_free.empty()) {
    *e = S->ev_free.back();
    S->ev_free.pop_back();
    return HJ_OK;
  }
  HJ_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
  return HJ_OK;
}

// A slot for request q: a free slot of the same problem, else a new one
// within the budget (destroying idle slots, least recently used first).
// Returns -1 in *slot when the request has to wait.
hj_status server_find_slot(hj_server *S, hj_server::Req &q, int *slot) {
  *slot = -1;
  int best = -1;
  for (size_t i = 0; i < S->slots.size(); ++i) {
    const auto &sl = S->slots[i];
    if (sl.g && !sl.busy && same_problem(sl.g, q.g, q.dyn)) {
      if (best < 0 || sl.last_use > S->slots[best].last_use) best = (int)i;
    }
  }
  if (best >= 0) {
    *slot = best;
    return HJ_OK;
  }
  int64_t need = slot_bytes_of(S, q.g);
  while (S->d.hbm_budget > 0 && S->slot_bytes + need > S->d.hbm_budget) {
    int victim = -1;
    for (size_t i = 0; i < S->slots.size(); ++i) {
      const auto &sl = S->slots[i];
      if (sl.g && !sl.busy && (victim < 0 || sl.last_use < S->slots[victim].last_use)) victim = (int)i;
    }
    if (victim < 0) return HJ_OK;  // everything is in use: wait
    hj_status st = hj_grid_destroy(S->slots[victim].g);
    if (st != HJ_OK) return st;
    S->slot_bytes -= S->slots[victim].bytes;
    S->slots[victim] = hj_server::Slot();
  }
  hj_grid *G = nullptr;
  hj_status st = hj_grid_create(&q.g, &q.dyn, &S->d.scheme, S->stream, &G);
  if (st != HJ_OK) return st;
  G->autotune_on = false;
  hj_server::Slot sl;
  sl.g = G;
  sl.bytes = need;
  S->slot_bytes += need;
  for (size_t i = 0; i < S->slots.size(); ++i)
    if (!S->slots[i].g) {
      S->slots[i] = sl;
      *slot = (int)i;
      return HJ_OK;
    }
  S->slots.push_back(sl);
  *slot = (int)S->slots.size() - 1;
  return HJ_OK;
}

hj_status server_admit(hj_server *S) {
  hj_status st;
  while (!S->queue.empty() && (int)S->running.size() < S->d.max_inflight) {
    const int64_t id = S->queue.front();
    hj_server::Req &q = S->reqs[id];
    int slot;
    if ((st = server_find_slot(S, q, &slot)) != HJ_OK) return st;
    if (slot < 0) break;  // head of the queue waits for memory
    hj_grid *G = S->slots[slot].g;
    if ((st = hj_set_target_cylinders(G, q.cx.data(), q.cy.data(), q.r.data(), (int32_t)q.cx.size())) != HJ_OK)
      return st;
    if ((st = ensure_dt(G)) != HJ_OK) return st;
    schedule(G, q.horizon, &q.n, &q.dt, &q.dt_last);
    S->slots[slot].busy = true;
    S->slots[slot].last_use = S->stats.ticks;
    q.slot = slot;
    q.k = 0;
    S->queue.pop_front();
    S->stats.admitted += 1;
    if (q.n == 0) {  // V = V0, already written with the target
      if ((st = server_event(S, &q.ev)) != HJ_OK) return st;
      HJ_HIP(hipEventRecord(q.ev, S->stream));
      q.state = 2;
    } else {
      q.state = 1;
      S->running.push_back(id);
    }
  }
  return HJ_OK;
}

// One step of request q at its step k + s on its own handle (the handle's
// stage kernel and chunking; the buffer roles follow the batch convention:
// V^0 = V0, V^k in v (k even) or w2 (k odd)).
template <typename T>
hj_status server_step_alone(hj_server *S, hj_server::Req &q, int64_t k) {
  hj_grid *G = S->slots[q.slot].g;
  const T *cur = k == 0 ? buf<const T>(G->v0) : ((k & 1) ? buf<const T>(G->w2) : buf<const T>(G->v));
  T *nxt = (k & 1) ? buf<T>(G->v) : buf<T>(G->w2);
  const double dt = k == q.n - 1 ? q.dt_last : q.dt;
  const int clamp = S->d.scheme.clamp == HJ_CLAMP_MIN_V0;
  if (S->d.scheme.integrator == HJ_EULER) return launch_one_stage<T>(G, cur, nullptr, nxt, hj::kPlain, clamp, dt);
  hj_status st = launch_one_stage<T>(G, cur, nullptr, buf<T>(G->w1), hj::kPlain, 0, dt);
  if (st != HJ_OK) return st;
  return launch_one_stage<T>(G, buf<const T>(G->w1), cur, nxt, hj::kAverage, clamp, dt);
}

template <typename T>
hj_status server_step(hj_server *S) {
  if (S->running.empty()) return HJ_OK;
  const int r = S->ring;
  S->ring = (r + 1) % hj_server::kRing;
  HJ_HIP(hipEventSynchronize(S->ring_ev[r]));  // this ring slot's previous launches are done
  // the requests that step this tick: all of them (sharing), or, in the
  // order small ones (least remaining work first) then large ones (first
  // submitted first), as many as it takes to fill the device -- except that
  // requests older than the age limit (since submission) go first, oldest
  // first, so that a stream of small requests cannot hold a large one back:
  // past the limit the order is first come, first served
  std::vector<int64_t> sel(S->running), wait;
  if (S->d.policy == HJ_SERVE_SMALL_FIRST) {
    const double now = host_seconds();
    const double age_s = (S->d.age_ms > 0 ? S->d.age_ms : kServerAgeMs) * 1e-3;
    auto npts = [&](int64_t id) { return S->slots[S->reqs[id].slot].g->npts; };
    auto key = [&](int64_t id) {
      const hj_server::Req &q = S->reqs[id];
      if (now - q.submitted_s >= age_s) return std::make_pair(0, id);
      const bool large = npts(id) >= kServerFillPoints;
      return std::make_pair(large ? 2 : 1, large ? id : npts(id) * (q.n - q.k));
    };
    std::stable_sort(sel.begin(), sel.end(), [&](int64_t x, int64_t y) { return key(x) < key(y); });
    size_t take = 0;
    for (int64_t pts = 0; take < sel.size() && pts < kServerFillPoints; ++take) pts += npts(sel[take]);
    wait.assign(sel.begin() + take, sel.end());
    sel.resize(take);
  }
  const int m = (int)sel.size();
  // longest remaining first, so the requests still stepping at step s of
  // this tick are a prefix of each group
  std::stable_sort(sel.begin(), sel.end(), [&](int64_t x, int64_t y) {
    const hj_server::Req &a = S->reqs[x], &b = S->reqs[y];
    return a.n - a.k > b.n - b.k;
  });
  const int64_t spt = S->d.steps_per_tick > 0 ? S->d.steps_per_tick : 4;
  // large grids fill the device alone and step on their own handle's
  // kernel; the others share one launch per stage and step -- unless a
  // small one is alone in the tick, when its own handle's kernel (the plane
  // kernel with its own chunking, where it fits) serves it better
  std::vector<int> big, small;
  for (int i = 0; i < m; ++i) {
    const hj_grid *G = S->slots[S->reqs[sel[i]].slot].g;
    (G->npts >= kServerAlonePoints ? big : small).push_back(i);
  }
  if (small.size() == 1) {
    big.push_back(small[0]);
    small.clear();
  }
  hj::BatchInst<T> *inst = static_cast<hj::BatchInst<T> *>(S->inst_host[r]);
  int32_t *tile_end = S->tile_host[r];
  // tile length: the server's, else x cut so that one launch over the small
  // requests has about kServerBlocks blocks
  int64_t row_blocks = 0;
  for (int i : small) {
    const hj_grid *G = S->slots[S->reqs[sel[i]].slot].g;
    int run = hj::run_length((int)sizeof(T), G->g.n[3]);
    row_blocks += ((int64_t)G->g.n[1] * G->g.n[2] * (G->g.n[3] / run) + hj::kStreamBlock - 1) / hj::kStreamBlock;
  }
  const int64_t want = row_blocks > 0 ? (kServerBlocks + row_blocks - 1) / row_blocks : 1;
  bool sg = false, ball = false;
  int64_t acc = 0;
  std::vector<int64_t> remain(m);
  for (int i = 0; i < m; ++i) {
    hj_server::Req &q = S->reqs[sel[i]];
    remain[i] = q.n - q.k;
  }
  for (size_t u = 0; u < small.size(); ++u) {
    hj_server::Req &q = S->reqs[sel[small[u]]];
    hj_grid *G = S->slots[q.slot].g;
    hj::BatchInst<T> &in = inst[u];
    memset(&in, 0, sizeof in);
    int chunks;
    if (S->d.x_planes > 0) {
      chunks = (G->g.n[0] + S->d.x_planes - 1) / S->d.x_planes;
    } else {
      int cap = G->g.n[0] / 4 > 1 ? G->g.n[0] / 4 : 1;
      chunks = (int)(want < cap ? want : cap);
    }
    in.a = batch_stream_args<T>(G, chunks);
    in.v0 = buf<const T>(G->v0);
    in.va = buf<T>(G->v);
    in.vb = buf<T>(G->w2);
    in.w1 = S->d.scheme.integrator == HJ_TVD_RK2 ? buf<T>(G->w1) : nullptr;
    in.dt = (T)q.dt;
    in.dt_last = (T)q.dt_last;
    in.steps = (int32_t)q.n;
    in.k = (int32_t)q.k;
    in.rk2 = S->d.scheme.integrator == HJ_TVD_RK2 ? 1 : 0;
    in.clamp = S->d.scheme.clamp == HJ_CLAMP_MIN_V0 ? 1 : 0;
    in.tiles = in.a.blocks_per_chunk * in.a.n_chunks;
    acc += in.tiles;
    tile_end[u] = (int32_t)acc;
    if (G->sig[0] != 0.0 || G->sig[1] != 0.0) sg = true;
    if (G->ball_mask != 0) ball = true;
  }
  if (acc >= ((int64_t)1 << 31)) return fail(HJ_ERR_UNSUPPORTED, "too many tiles in one tick");
  if (!small.empty()) {
    HJ_HIP(hipMemcpyAsync(S->tile_dev[r], tile_end, small.size() * sizeof(int32_t), hipMemcpyHostToDevice, S->stream));
    HJ_HIP(hipMemcpyAsync(S->inst_dev[r], inst, small.size() * sizeof(hj::BatchInst<T>), hipMemcpyHostToDevice,
                          S->stream));
  }
  const hj::BatchInst<T> *di = static_cast<const hj::BatchInst<T> *>(S->inst_dev[r]);
  const int stages = S->d.scheme.integrator == HJ_TVD_RK2 ? 2 : 1;
  const int64_t nsteps = remain[0] < spt ? remain[0] : spt;
  int act = (int)small.size();
  for (int64_t s = 0; s < nsteps; ++s) {
    // requests that took their last step at s - 1: their V is final once
    // the launches enqueued so far have run
    for (int i = 0; i < m; ++i)
      if (remain[i] == s) {
        hj_server::Req &q = S->reqs[sel[i]];
        hj_status st = server_event(S, &q.ev);
        if (st != HJ_OK) return st;
        HJ_HIP(hipEventRecord(q.ev, S->stream));
      }
    while (act > 0 && remain[small[act - 1]] <= s) --act;
    for (int st = 0; st < stages && act > 0; ++st)
      HJ_HIP(hj::launch_multi<T>(di, S->tile_dev[r], act, tile_end[act - 1], (int)(-1 - s), st, S->d.scheme.deriv,
                                 sg, ball, S->stream));
    for (int i : big)
      if (remain[i] > s) {
        hj_server::Req &q = S->reqs[sel[i]];
        hj_status st = server_step_alone<T>(S, q, q.k + s);
        if (st != HJ_OK) return st;
      }
  }
  HJ_HIP(hipEventRecord(S->ring_ev[r], S->stream));
  // advance; retire the requests that took their last step
  std::vector<int64_t> still;
  for (int i = 0; i < m; ++i) {
    const int64_t id = sel[i];
    hj_server::Req &q = S->reqs[id];
    q.k += remain[i] < nsteps ? remain[i] : nsteps;
    if (q.k < q.n) {
      still.push_back(id);
      continue;
    }
    hj_grid *G = S->slots[q.slot].g;
    if (q.n & 1) {  // V^n is in w2
      void *t = G->v;
      G->v = G->w2;
      G->w2 = t;
    }
    if (!q.ev) {  // finished at the last step of the tick
      hj_status st = server_event(S, &q.ev);
      if (st != HJ_OK) return st;
      HJ_HIP(hipEventRecord(q.ev, S->stream));
    }
    q.state = 2;
  }
  still.insert(still.end(), wait.begin(), wait.end());
  S->running.swap(still);
  return HJ_OK;
}

hj_status check_server(hj_server *S) {
  if (!S) return fail(HJ_ERR_INVALID_ARG, "null server");
  return HJ_OK;
}

void server_counts(hj_server *S) {
  S->stats.running = (int32_t)S->running.size();
  S->stats.queued = (int32_t)S->queue.size();
  int32_t n = 0;
  for (auto &sl : S->slots)
    if (sl.g) ++n;
  S->stats.slots = n;
  S->stats.slot_bytes = S->slot_bytes;
}

hj_status server_release_slot(hj_server *S, int64_t id) {
  auto it = S->reqs.find(id);
  hj_server::Req &q = it->second;
  S->slots[q.slot].busy = false;
  S->slots[q.slot].last_use = S->stats.ticks;
  if (q.ev) S->ev_free.push_back(q.ev);
  S->reqs.erase(it);
  return HJ_OK;
}

}  // namespace

extern "C" {

hj_status hj_server_create(const hj_server_desc *desc, void *hip_stream, hj_server **out) {
  if (!out) return fail(HJ_ERR_INVALID_ARG, "null output handle pointer");
  *out = nullptr;
  if (!desc) return fail(HJ_ERR_INVALID_ARG, "null server description");
  if (desc->max_inflight < 1 || desc->max_inflight > hj::kMaxBatch)
    return fail(HJ_ERR_INVALID_ARG, "max_inflight must be 1..%d", hj::kMaxBatch);
  if (desc->hbm_budget < 0 || desc->x_planes < 0 || desc->steps_per_tick < 0 || !(desc->age_ms >= 0.0))
    return fail(HJ_ERR_INVALID_ARG, "negative budget, tile or steps per tick");
  if (desc->policy != HJ_SERVE_SMALL_FIRST && desc->policy != HJ_SERVE_SHARE)
    return fail(HJ_ERR_INVALID_ARG, "unknown server policy %d", desc->policy);
  const hj_scheme_desc &sc = desc->scheme;
  if ((sc.deriv != HJ_UPWIND1 && sc.deriv != HJ_ENO2) || (sc.integrator != HJ_EULER && sc.integrator != HJ_TVD_RK2) ||
      (sc.precision != HJ_F32 && sc.precision != HJ_F64) || (sc.clamp != HJ_CLAMP_NONE && sc.clamp != HJ_CLAMP_MIN_V0) ||
      !(sc.cfl > 0.0 && sc.cfl <= 1.0))
    return fail(HJ_ERR_INVALID_ARG, "invalid scheme");
  if (sc.alpha_mode != HJ_ALPHA_STATE) return fail(HJ_ERR_UNSUPPORTED, "servers need the state-bound alpha");
  hj_server *S = new (std::nothrow) hj_server;
  if (!S) return fail(HJ_ERR_OUT_OF_MEMORY, "host allocation failed");
  S->d = *desc;
  S->stream = static_cast<hipStream_t>(hip_stream);
  S->elem = sc.precision == HJ_F32 ? 4 : 8;
  size_t inst_bytes = (size_t)hj::kMaxBatch * (S->elem == 4 ? sizeof(hj::BatchInst<float>) : sizeof(hj::BatchInst<double>));
  hipError_t e = hipGetDevice(&S->device);
  for (int i = 0; i < hj_server::kRing && e == hipSuccess; ++i) {
    e = hipMalloc(&S->inst_dev[i], inst_bytes);
    if (e == hipSuccess) e = hipHostMalloc(&S->inst_host[i], inst_bytes, 0);
    if (e == hipSuccess) e = hipMalloc((void **)&S->tile_dev[i], hj::kMaxBatch * sizeof(int32_t));
    if (e == hipSuccess) e = hipHostMalloc((void **)&S->tile_host[i], hj::kMaxBatch * sizeof(int32_t), 0);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->ring_ev[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(S->ring_ev[i], S->stream);
  }
  if (e != hipSuccess) {
    server_free(S);
    delete S;
    return fail(e == hipErrorOutOfMemory ? HJ_ERR_OUT_OF_MEMORY : HJ_ERR_DEVICE, "hj_server_create: %s",
                hipGetErrorString(e));
  }
  *out = S;
  return HJ_OK;
}

hj_status hj_server_destroy(hj_server *S) {
  if (!S) return HJ_OK;
  (void)hipSetDevice(S->device);
  (void)hipStreamSynchronize(S->stream);
  server_free(S);
  delete S;
  return HJ_OK;
}

hj_status hj_server_submit(hj_server *S, const hj_grid_desc *grid, const hj_dynamics_desc *dyn, const double *cx,
                           const double *cy, const double *r, int32_t m, double horizon, int64_t *id) {
  hj_status st = check_server(S);
  if (st != HJ_OK) return st;
  if (!id) return fail(HJ_ERR_INVALID_ARG, "null id output");
  if (!isfinite(horizon) || horizon < 0) return fail(HJ_ERR_INVALID_ARG, "horizon must be finite and >= 0");
  if ((st = validate(grid, dyn, &S->d.scheme)) != HJ_OK) return st;
  if (!cx || !cy || !r || m < 1) return fail(HJ_ERR_INVALID_ARG, "need at least one obstacle");
  if (bit(grid->periodic_mask, 0) || bit(grid->periodic_mask, 1))
    return fail(HJ_ERR_INVALID_ARG, "cylinder targets need open x and y axes");
  if (!bit(grid->periodic_mask, 3)) return fail(HJ_ERR_UNSUPPORTED, "serving needs a periodic theta axis");
  for (int o = 0; o < m; ++o)
    if (!isfinite(cx[o]) || !isfinite(cy[o]) || !isfinite(r[o]) || r[o] < 0)
      return fail(HJ_ERR_INVALID_ARG, "obstacle %d: need finite centre and radius >= 0", o);
  if (S->d.hbm_budget > 0 && slot_bytes_of(S, *grid) > S->d.hbm_budget)
    return fail(HJ_ERR_OUT_OF_MEMORY, "one grid of this size exceeds the server's memory budget");
  hj_server::Req q;
  q.g = *grid;
  q.dyn = *dyn;
  q.cx.assign(cx, cx + m);
  q.cy.assign(cy, cy + m);
  q.r.assign(r, r + m);
  q.horizon = horizon;
  q.submitted_s = host_seconds();
  int64_t nid = S->next_id++;
  S->reqs[nid] = q;
  S->queue.push_back(nid);
  S->stats.submitted += 1;
  *id = nid;
  return HJ_OK;
}

hj_status hj_server_tick(hj_server *S, int32_t *running) {
  hj_status st = check_server(S);
  if (st != HJ_OK) return st;
  HJ_HIP(hipSetDevice(S->device));
  if ((st = server_admit(S)) != HJ_OK) return st;
  st = S->elem == 4 ? server_step<float>(S) : server_step<double>(S);
  if (st != HJ_OK) return st;
  S->stats.ticks += 1;
  if (running) *running = (int32_t)S->running.size();
  return HJ_OK;
}

hj_status hj_server_poll(hj_server *S, int64_t *ids, int32_t cap, int32_t *n) {
  hj_status st = check_server(S);
  if (st != HJ_OK) return st;
  if (!n || (cap > 0 && !ids)) return fail(HJ_ERR_INVALID_ARG, "null output");
  *n = 0;
  for (auto &kv : S->reqs) {
    hj_server::Req &q = kv.second;
    if (q.state == 2) {
      hipError_t e = hipEventQuery(q.ev);
      if (e == hipSuccess) {
        q.state = 3;
        S->stats.completed += 1;
      } else if (e != hipErrorNotReady) {
        return fail(HJ_ERR_DEVICE, "hj_server_poll: %s", hipGetErrorString(e));
      }
    }
    if (q.state == 3 && *n < cap) ids[(*n)++] = kv.first;
  }
  return HJ_OK;
}

hj_status hj_server_take(hj_server *S, int64_t id, void *out, int32_t dtype, int32_t where) {
  hj_status st = check_server(S);
  if (st != HJ_OK) return st;
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return fail(HJ_ERR_INVALID_ARG, "unknown request %lld", (long long)id);
  if (it->second.state != 3) return fail(HJ_ERR_NOT_READY, "request %lld is not complete", (long long)id);
  if (out && (st = hj_get_value(S->slots[it->second.slot].g, out, dtype, where)) != HJ_OK) return st;
  return server_release_slot(S, id);
}

hj_status hj_server_get_stats(hj_server *S, hj_server_stats *out) {
  hj_status st = check_server(S);
  if (st != HJ_OK) return st;
  if (!out) return fail(HJ_ERR_INVALID_ARG, "null output");
  server_counts(S);
  *out = S->stats;
  return HJ_OK;
}

}  // extern "C"
