// hj_internal.h -- kernel argument blocks and launcher declarations shared by
// the ABI layer (hj_abi.hip) and the kernels (hj_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hj {

enum Deriv { kUpwind1 = 0, kEno2 = 1 };

// How a stage combines its Lax-Friedrichs right-hand side L(Vs):
//   kPlain: out = Vs + dt L(Vs)                 (Euler; TVD-RK2 stage 1)
//   kAverage: out = (Vn + Vs + dt L(Vs)) / 2     (TVD-RK2 stage 2)
enum StageMode { kPlain = 0, kAverage = 1 };

// The Hamiltonian of every supported dynamics, written in separable form
// (see the kernels for the derivation):
//   H(z, p) = bx(v,th) px + by(v,th) py + bv pv + bth pth
//           + sum_d sig_d |p_d| + sig_ball |p_S|_2
// and the dissipation coefficients alpha = (ax(v,th), ay(v,th), av, ath).
// Per-(v, theta) values live in a table of four arrays (bx, by, ax, ay), each
// Nv * Ntheta long, index k * Ntheta + l.
template <typename T>
struct StageArgs {
  const T *vs;   // stencil input: V^n (Euler, stage 1) or V^1 (stage 2)
  const T *vn;   // V^n for the stage-2 average (unused in kPlain)
  const T *v0;   // target, for the clamp (unused without clamp)
  T *out;
  const T *lut;  // bx | by | ax | ay, each n[2] * n[3] values
  const T *th;   // alpha_theta | sig_theta, each n[2] values (theta axis per v)
  int32_t n[4];
  int64_t st[4];  // C-order strides of the external layout
  uint32_t periodic_mask;
  T inv_h[4];
  T bv, bth, av, ath;
  T sig[4];
  T sig_ball;
  uint32_t ball_mask;
  T dt;
  int32_t mode;
  int32_t clamp;
  int64_t npts;
  const int32_t *skip;  // when non-null and *skip != 0 the launch does nothing
  // Derivative-range pass: 0 = range of the central derivative (p- + p+) / 2
  // (Algorithm 1), 1 = range of both one-sided derivatives
  int32_t range_onesided;
};

// The streaming stage kernel (see hj_kernels.hip).  Each thread owns a run
// of R consecutive theta nodes at one (y, v) and sweeps a chunk of x planes.
// The right-hand side is written per axis as
//   L_d = kp_d p+_d + km_d p-_d + sg_d |p+_d + p-_d|
// with unscaled one-sided differences p' = h p:
//   kp = (b + alpha) / (2h), km = (b - alpha) / (2h), sg = sig / (2h).
// kp, km of x and y vary with (v, theta) (table `coef`: kp_x | km_x | kp_y |
// km_y, each n[2] * n[3]); those of theta vary with v (the steering car
// turns at most |v| tan(delta_max) / L; table `coef_th`), those of v are
// uniform.
template <typename T>
struct StreamArgs {
  const T *vs;
  const T *vn;
  const T *v0;
  T *out;
  const T *coef;
  const T *v0xy;  // target as an n[0] x n[1] table (constant over v, theta), or null
  int32_t n[4];
  uint32_t periodic_mask;
  int32_t plane;           // n[1] * n[2] * n[3]: stride of x
  int32_t row;             // n[2] * n[3]: stride of y
  int32_t run;             // R, theta nodes per thread (run_length)
  int32_t runs_per_row;    // n[3] / R
  int32_t slab_runs;       // n[1] * n[2] * runs_per_row
  int32_t blocks_per_chunk;
  int32_t chunk_len;       // x planes per block
  int32_t n_chunks;
  int32_t v_seg;     // plane kernel: v rows per block (n[2] unless the plane is split)
  int32_t n_seg;     // plane kernel: v segments (1: the whole plane in one block)
  const T *coef_th;  // kp_theta | km_theta | sg_theta, each n[2] values (per v)
  T kp_v, km_v;
  T sg[4];
  T half_inv_h[4];  // 1 / (2 h_d), for the ball term
  T sig_ball;
  uint32_t ball_mask;
  T dt;
  int32_t mode;
  int32_t clamp;
  const int32_t *skip;  // when non-null and *skip != 0 the launch does nothing
  // Plane kernel, last stage of a step: when non-null, the largest change of
  // a node, max |out - V^n| in FP64 (NaN as infinity), is folded in with an
  // atomic max of its bits (non-negative doubles order as their bits)
  unsigned long long *eps;
  // Range pass (plane kernel, RANGE instance): kRangeSlots sets of keys of
  // the per-axis extremes of the derivatives (see launch_deriv_range): of
  // the central derivative (p- + p+) / 2 (Algorithm 1), or of both one-sided
  // derivatives when range_onesided is set
  unsigned long long *range;
  int32_t range_onesided;
  // Plane kernel: 0 = chunk mode (one block per (x chunk, v segment, y row));
  // else this many blocks share the ny * nx row-planes of a whole-plane grid
  // equally in row-major order (blocks may span two or more rows)
  int32_t span;
  // Plane kernel, chunk mode: y rows per block, 1 or 2 (2: the block holds
  // rows 2u and 2u + 1 of its v segment, n[1] even; blocks_per_chunk is
  // then n[1] / 2 * n_seg)
  int32_t rows;
};

constexpr int kStreamBlock = 256;

// Run length (theta nodes per thread) of the streaming and plane kernels:
// the longest of 4 (FP32; 2 in FP64), 2 and 1 that divides N_theta, so runs
// are 16-byte, 8-byte or single-element loads.
inline int run_length(int elem, int nth) {
  int r = elem == 4 ? 4 : 2;
  while (r > 1 && nth % r != 0) r /= 2;
  return r;
}

template <typename T>
hipError_t launch_stream(const StreamArgs<T> &a, int deriv, bool ball, hipStream_t s);

// The plane kernel: one block per (y row, x chunk) holds the whole
// (v, theta) plane of the current x in LDS; it needs n[2] * n[3] / R <= 768
// runs and 2 n[2] n[3] values of LDS.  A larger plane is split along v into
// n_seg segments of v_seg rows (v_seg * n[3] / R <= 768 runs), each block
// holding its segment and two halo rows per side: 2 (v_seg + 4) n[3] values.
// blocks_per_chunk = n[1] * n_seg (segment-major, y fastest).
constexpr int kPlaneMaxThreads = 768;
// Runs of 3 theta nodes (FP32, whole planes only): each run takes a 4-element
// LDS slot, and a block may hold up to 1024 runs (16 waves).
constexpr int kPlaneMaxThreads3 = 1024;
constexpr int kPlaneMaxLdsBytes = 64 * 1024;
constexpr int kPlaneMinSegRows = 4;  // a split plane keeps at least this many rows per block

template <typename T>
hipError_t launch_plane(const StreamArgs<T> &a, int deriv, bool ball, hipStream_t s);

// ---- batched solves -------------------------------------------------------
// Instance j of a batch: the streaming-kernel description of its grid (the
// per-phase fields vs, vn, out, dt, mode and clamp are filled in by the
// kernels) and its time schedule.  Step k reads V^k and writes V^(k+1):
// V^0 is the target V0 itself, V^k for k >= 1 lives in va (k even) or vb
// (k odd).  Stage 1 of a TVD-RK2 step writes w1.
template <typename T>
struct BatchInst {
  StreamArgs<T> a;
  const T *v0;
  T *va, *vb, *w1;
  T dt, dt_last;   // steps 0 .. n-2 use dt, step n-1 dt_last
  int32_t steps;   // n
  int32_t rk2;     // 1: TVD-RK2 (two phases per step), 0: Euler (one)
  int32_t clamp;   // min(V0, .) after the last stage of a step
  int32_t tiles;   // blocks of one phase: a.blocks_per_chunk * a.n_chunks
  int32_t k;       // the instance's own step, for launches given k < 0
};

constexpr int kMaxBatch = 256;

// Device state of the persistent batch kernel: the next work item, an error
// flag (a dependency wait ran out of spins) and, per instance, the number of
// its tiles completed so far (over all phases).
struct BatchQueue {
  int32_t next;
  int32_t error;
  int32_t pad[2];
  int32_t done[kMaxBatch];
};

// The persistent kernel's work list: phase p (step p / phases_per_step,
// stage p % phases_per_step) holds the tiles of its first active[p]
// instances (instances are sorted by step count, longest first), items
// start[p] .. start[p+1]-1; tile_end[j] = tiles of instances 0..j.
template <typename T>
struct PersistArgs {
  const BatchInst<T> *inst;
  const int32_t *tile_end;
  const int32_t *start;   // nphase + 1 entries
  const int32_t *active;  // nphase entries
  BatchQueue *queue;
  int32_t nphase;
  int32_t phases_per_step;
  int64_t spin_limit;     // polls of a dependency before giving up
};

// One launch of phase (k, stage) over the first ninst instances (their
// tiles are blocks 0 .. tile_end[ninst-1]-1, XCD-contiguous); k < 0: each
// instance at its own step inst[j].k + (-1 - k).
template <typename T>
hipError_t launch_multi(const BatchInst<T> *inst, const int32_t *tile_end, int ninst, int blocks, int k, int stage,
                        int deriv, bool sg, bool ball, hipStream_t s);

// The batched plane kernel: the same launches with each instance's blocks
// running the plane kernel on its grid (inst[j].a a plane description:
// whole planes, or v segments, with chunk_len x planes per block), in
// blocks of `threads` work-items (a multiple of 64, at least the largest
// instance's runs) with `lds` bytes of LDS (at least the largest instance's).
template <typename T>
hipError_t launch_plane_multi(const BatchInst<T> *inst, const int32_t *tile_end, int ninst, int blocks, int threads,
                              size_t lds, int k, int stage, int deriv, bool sg, bool ball, hipStream_t s);

// Whether the plane description `a` runs in the batched plane kernel (run
// lengths 2 and, FP32, 3 and 4 -- a plane step of one theta node per
// work-item costs about as much as one of four, so runs of one are left to
// the streaming tiles; at most kPlaneMaxThreads runs per block; chunk mode),
// and the work-items and LDS bytes of its blocks.
template <typename T>
bool plane_multi_fits(const StreamArgs<T> &a, int *threads, size_t *lds);

// The whole batch in one launch of `blocks` persistent blocks.
template <typename T>
hipError_t launch_persistent(const PersistArgs<T> &p, int blocks, int deriv, bool sg, bool ball, hipStream_t s);

// Resident blocks per CU of the persistent kernel (occupancy).
template <typename T>
int persistent_blocks_per_cu(int deriv, bool sg, bool ball);

// queue->next = queue->error = 0, done[0..m) = 0 (a kernel, so that the
// sequence can be captured in a graph).
hipError_t launch_batch_reset(BatchQueue *queue, int m, hipStream_t s);

// ---- Algorithm 1's derivative range -----------------------------------------
// kRangeSlots sets of eight keys: set k holds, over the blocks with
// blockIdx % kRangeSlots == k, in keys[8k + d] / keys[8k + 4 + d] the
// order-preserving keys of the smallest / largest one-sided derivative (p-
// or p+) on axis d over the nodes of a.vs; the caller reduces the sets (the
// blocks' atomics spread over the sets instead of meeting on eight words).
constexpr int kRangeSlots = 64;
// The same keys from the plane kernel's traversal (grids the plane kernel
// runs; a.vs = V, a.range = the key sets)
template <typename T>
hipError_t launch_plane_range(StreamArgs<T> a, int deriv, hipStream_t s);
template <typename T>
hipError_t launch_deriv_range(const StageArgs<T> &a, int deriv, unsigned long long *keys, hipStream_t s);

// ---- convergence mode ----------------------------------------------------
// acc = max over i < n of |a[i] - b[i]| as the bit pattern of a non-negative
// double (NaN counts as +inf); nothing when *skip.
template <typename T>
hipError_t launch_delta_max(const T *a, const T *b, int64_t n, unsigned long long *acc, const int32_t *skip,
                            hipStream_t s);

// state[0] = stopped, state[1] = step count at the stop.  Unless stopped:
// eps_log[slot] = eps = acc, acc = 0, and eps < threshold stops after step k.
hipError_t launch_converge_check(unsigned long long *acc, double threshold, int32_t *state, double *eps_log, int slot,
                                 int64_t k, hipStream_t s);

// state[0] = state[1] = 0, acc = 0 (a kernel, graph-safe).
hipError_t launch_converge_reset(unsigned long long *acc, int32_t *state, hipStream_t s);

// ---- optimal control at arbitrary states (eq (9)) -------------------------
template <typename T>
struct ControlArgs {
  const T *v;
  int32_t n[4];
  uint32_t periodic_mask;
  double lo[4], hi[4], h[4];
  const double *states;  // m x 4
  int64_t m;
  double *controls;  // m x 2
  double *values;    // m, may be null
  double *grads;     // m x 4, may be null
  int32_t steer;     // 0: (a, w) car, 1: (a, delta) steering car
  double a_max, turn_max;
};

template <typename T>
hipError_t launch_control(const ControlArgs<T> &a, hipStream_t s);

constexpr int kMaxCylindersPerLaunch = 32;

template <typename T>
struct CylinderArgs {
  T *v0;
  T *v;  // also written (V := V0); may equal nullptr
  T *v0xy;  // the n0 x n1 table of the target
  int32_t n0, n1;
  int64_t plane;  // nodes per (x, y) pair: n[2] * n[3]
  T lo0, h0, lo1, h1;
  int32_t m;
  int32_t combine;  // 0: overwrite, 1: min with the existing V0
  T cx[kMaxCylindersPerLaunch], cy[kMaxCylindersPerLaunch], r[kMaxCylindersPerLaunch];
};

template <typename T>
hipError_t launch_stage(const StageArgs<T> &a, int deriv, bool ball, hipStream_t s);

template <typename T>
hipError_t launch_cylinders(const CylinderArgs<T> &a, hipStream_t s);

// alpha_max[0..1] = max over the table of ax, ay (FP64); [2], [3] = av, ath.
hipError_t launch_alpha_max(const double *ax, const double *ay, int64_t m, double av, double ath,
                            double *alpha_max, hipStream_t s);

// dst[i] = (To)src[i]
template <typename To, typename Ti>
hipError_t launch_cast(To *dst, const Ti *src, int64_t n, hipStream_t s);

template <typename T>
hipError_t launch_copy(T *dst, const T *src, int64_t n, hipStream_t s);

// flag[0] = 1 if any of the n values is NaN or infinite (flag cleared first).
template <typename T>
hipError_t launch_nonfinite(const T *src, int64_t n, int32_t *flag, hipStream_t s);

}  // namespace hj
