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
};

// The streaming stage kernel (see hj_kernels.hip).  Each thread owns a run
// of R consecutive theta nodes at one (y, v) and sweeps a chunk of x planes.
// The right-hand side is written per axis as
//   L_d = kp_d p+_d + km_d p-_d + sg_d |p+_d + p-_d|
// with unscaled one-sided differences p' = h p:
//   kp = (b + alpha) / (2h), km = (b - alpha) / (2h), sg = sig / (2h).
// kp, km of x and y vary with (v, theta) (table `coef`: kp_x | km_x | kp_y |
// km_y, each n[2] * n[3]); those of v and theta are uniform.
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
  int32_t runs_per_row;    // n[3] / R
  int32_t slab_runs;       // n[1] * n[2] * runs_per_row
  int32_t blocks_per_chunk;
  int32_t chunk_len;       // x planes per block
  int32_t n_chunks;
  T kp_v, km_v, kp_th, km_th;
  T sg[4];
  T half_inv_h[4];  // 1 / (2 h_d), for the ball term
  T sig_ball;
  uint32_t ball_mask;
  T dt;
  int32_t mode;
  int32_t clamp;
};

constexpr int kStreamBlock = 256;

// Run length of the streaming kernel per precision (16-byte vector loads).
template <typename T>
constexpr int stream_run() {
  return sizeof(T) == 4 ? 4 : 2;
}

template <typename T>
hipError_t launch_stream(const StreamArgs<T> &a, int deriv, bool ball, hipStream_t s);

// The plane kernel: one block per (y row, x chunk) holds the whole
// (v, theta) plane of the current x in LDS; it needs n[2] * n[3] / R <= 1024
// runs and 2 n[2] n[3] values of LDS.  Uses blocks_per_chunk = n[1].
constexpr int kPlaneMaxThreads = 1024;
constexpr int kPlaneMaxLdsBytes = 64 * 1024;

template <typename T>
hipError_t launch_plane(const StreamArgs<T> &a, int deriv, bool ball, hipStream_t s);

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
