// hj_kernels.hip -- gfx950 kernels of the HJ reachability time step.
//
//   stage_generic  one Lax-Friedrichs stage at every grid node (Algorithm 2,
//                  one sweep): one-sided derivatives per axis (eq (5) or
//                  second-order ENO), Hamiltonian with the optimal bang-bang
//                  inputs, dissipation, explicit update, optional clamp.
//   cylinders      target V0 of eq (7) for a union of cylinders, written to
//                  V0 and V.
//   alpha_max      FP64 max-reduction of the dissipation coefficients for the
//                  CFL step (Algorithm 1, step-bound lines).
//   cast/copy/nonfinite  layout-preserving helpers.
//
// Memory-bound stencil: no matrix cores.  wave64 throughout.

#include <float.h>
#include <math.h>

#include "hj_internal.h"

namespace hj {

namespace {

constexpr int kNumXcd = 8;

// Work-groups are handed to the 8 XCDs round-robin (block b runs on XCD
// b % 8).  Renumber them so that each XCD receives one contiguous range of
// logical blocks: neighbouring tiles then share that XCD's L2.
__device__ inline int64_t xcd_logical_block(int64_t b, int64_t nblocks) {
  int64_t q = nblocks / kNumXcd, r = nblocks % kNumXcd;
  int64_t x = b % kNumXcd, local = b / kNumXcd;
  int64_t start = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  return start + local;
}

template <typename T>
__device__ inline T tabs(T x) {
  return x < T(0) ? -x : x;
}

// Value `o` nodes away from node i (0 <= i < n) along an axis of stride s:
// on the grid, wrapped on a periodic axis, else linearly extrapolated from
// the two end nodes (ghost k layers out = V_end + k (V_end - V_next)).
template <typename T>
__device__ inline T axis_value(const T *__restrict__ v, int64_t p, int i, int o, int n, int64_t s,
                               bool periodic) {
  int q = i + o;
  if (q >= 0 && q < n) return v[p + (int64_t)o * s];
  if (periodic) {
    int qq = q < 0 ? q + n : q - n;
    return v[p + (int64_t)(qq - i) * s];
  }
  if (q < 0) {
    T e = v[p - (int64_t)i * s], nx = v[p - (int64_t)(i - 1) * s];
    return e + T(-q) * (e - nx);
  }
  T e = v[p + (int64_t)(n - 1 - i) * s], nx = v[p + (int64_t)(n - 2 - i) * s];
  return e + T(q - (n - 1)) * (e - nx);
}

// Second difference Q_j = V_{j+1} - 2 V_j + V_{j-1}, evaluated as
// (V_{j+1} - 2 V_j) + V_{j-1}: the doubling is exact, so fused or not this is
// two roundings, and equal inputs give equal Q (and equal ENO choices).
template <typename T>
__device__ inline T second_diff(T vm, T v0, T vp) {
  return (vp - T(2) * v0) + vm;
}

// One-sided derivatives from the window w[0..4] = V_{i-2..i+2} (upwind uses
// w[1..3]).  ENO2: the second-order correction takes the smaller-magnitude
// second difference on the side of the derivative (ties: the left one).
template <typename T, int DERIV>
__device__ inline void one_sided(const T (&w)[5], T inv_h, T &pm, T &pp) {
  if (DERIV == kUpwind1) {
    pm = (w[2] - w[1]) * inv_h;
    pp = (w[3] - w[2]) * inv_h;
  } else {
    T ql = second_diff(w[0], w[1], w[2]);
    T qm = second_diff(w[1], w[2], w[3]);
    T qr = second_diff(w[2], w[3], w[4]);
    T cm = tabs(ql) <= tabs(qm) ? ql : qm;
    T cp = tabs(qm) <= tabs(qr) ? qm : qr;
    pm = ((w[2] - w[1]) + T(0.5) * cm) * inv_h;
    pp = ((w[3] - w[2]) - T(0.5) * cp) * inv_h;
  }
}

// Lax-Friedrichs right-hand side from the one-sided derivatives.
//
// Every supported dynamics is affine in its inputs with box (or, for the
// test dynamics, ball) bounds, so max_u min_d p.f splits per axis:
//   - an uncontrolled velocity term b_d contributes b_d p_d;
//   - a maximising input bounded by s on axis d contributes +s |p_d|;
//   - a minimising one (the disturbance) contributes -s |p_d|;
//   - a ball-bounded input contributes +-s |p_S|_2.
// The dissipation adds alpha_d (p+ - p-) / 2 with alpha_d the bound on |f_d|.
template <typename T, bool BALL>
__device__ inline T lf_rhs(const T (&pm)[4], const T (&pp)[4], T bx, T by, T ax, T ay,
                           const StageArgs<T> &a) {
  T pb[4], hd[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    pb[d] = T(0.5) * (pp[d] + pm[d]);
    hd[d] = T(0.5) * (pp[d] - pm[d]);
  }
  T L = bx * pb[0] + by * pb[1] + a.bv * pb[2] + a.bth * pb[3];
#pragma unroll
  for (int d = 0; d < 4; ++d) L += a.sig[d] * tabs(pb[d]);
  L += ax * hd[0] + ay * hd[1] + a.av * hd[2] + a.ath * hd[3];
  if (BALL) {
    T s2 = T(0);
#pragma unroll
    for (int d = 0; d < 4; ++d)
      if ((a.ball_mask >> d) & 1u) s2 += pb[d] * pb[d];
    L += a.sig_ball * sqrt(s2);
  }
  return L;
}

template <typename T>
__device__ inline T finish(const StageArgs<T> &a, int64_t p, T vs, T L) {
  T r = vs + a.dt * L;
  if (a.mode == kAverage) r = T(0.5) * (a.vn[p] + r);
  if (a.clamp) {
    T t = a.v0[p];
    r = t < r ? t : r;
  }
  return r;
}

// One thread per node, neighbours read straight from global memory (L1/L2
// serve the reuse).  Works for every grid shape.
template <typename T, int DERIV, bool BALL>
__global__ __launch_bounds__(256) void stage_generic(StageArgs<T> a) {
  int64_t blk = xcd_logical_block(blockIdx.x, gridDim.x);
  int64_t p = blk * 256 + threadIdx.x;
  if (p >= a.npts) return;
  int idx[4];
  {
    int64_t q = p;
    idx[3] = (int)(q % a.n[3]);
    q /= a.n[3];
    idx[2] = (int)(q % a.n[2]);
    q /= a.n[2];
    idx[1] = (int)(q % a.n[1]);
    idx[0] = (int)(q / a.n[1]);
  }
  const T *__restrict__ v = a.vs;
  T pm[4], pp[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    T w[5];
    bool per = (a.periodic_mask >> d) & 1u;
    const int R = DERIV == kUpwind1 ? 1 : 2;
#pragma unroll
    for (int o = -2; o <= 2; ++o)
      w[o + 2] = (o < -R || o > R) ? T(0) : axis_value(v, p, idx[d], o, a.n[d], a.st[d], per);
    one_sided<T, DERIV>(w, a.inv_h[d], pm[d], pp[d]);
  }
  int64_t c = (int64_t)idx[2] * a.n[3] + idx[3];
  int64_t m = (int64_t)a.n[2] * a.n[3];
  T bx = a.lut[c], by = a.lut[m + c], ax = a.lut[2 * m + c], ay = a.lut[3 * m + c];
  T L = lf_rhs<T, BALL>(pm, pp, bx, by, ax, ay, a);
  a.out[p] = finish(a, p, v[p], L);
}

// Target: one block per (x, y) pair computes the distance once and writes
// it over the whole (v, theta) plane.
template <typename T>
__global__ __launch_bounds__(256) void cylinders_kernel(CylinderArgs<T> a) {
  int ij = blockIdx.x;
  int i = ij / a.n1, j = ij % a.n1;
  T x = a.lo0 + T(i) * a.h0, y = a.lo1 + T(j) * a.h1;
  T best = INFINITY;
  for (int o = 0; o < a.m; ++o) {
    T dx = x - a.cx[o], dy = y - a.cy[o];
    T dist = sqrt(dx * dx + dy * dy) - a.r[o];
    best = dist < best ? dist : best;
  }
  int64_t base = (int64_t)ij * a.plane;
  for (int64_t q = threadIdx.x; q < a.plane; q += blockDim.x) {
    T val = best;
    if (a.combine) {
      T old = a.v0[base + q];
      val = old < val ? old : val;
    }
    a.v0[base + q] = val;
    if (a.v) a.v[base + q] = val;
  }
}

__device__ inline double wave_max(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    double y = __shfl_xor(x, off, 64);
    x = y > x ? y : x;
  }
  return x;
}

// Single work-group FP64 max over the table (a few thousand entries):
// per-lane max, wave64 butterfly over shuffles, then across the 4 waves in
// LDS.  Deterministic (max is order-free).
__global__ __launch_bounds__(256) void alpha_max_kernel(const double *__restrict__ ax,
                                                        const double *__restrict__ ay, int64_t m,
                                                        double av, double ath,
                                                        double *__restrict__ out) {
  __shared__ double part[2][4];
  double mx = 0.0, my = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
    mx = ax[i] > mx ? ax[i] : mx;
    my = ay[i] > my ? ay[i] : my;
  }
  mx = wave_max(mx);
  my = wave_max(my);
  int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) {
    part[0][wave] = mx;
    part[1][wave] = my;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double rx = part[0][0], ry = part[1][0];
    for (int w = 1; w < 4; ++w) {
      rx = part[0][w] > rx ? part[0][w] : rx;
      ry = part[1][w] > ry ? part[1][w] : ry;
    }
    out[0] = rx;
    out[1] = ry;
    out[2] = av;
    out[3] = ath;
  }
}

template <typename To, typename Ti>
__global__ __launch_bounds__(256) void cast_kernel(To *__restrict__ dst, const Ti *__restrict__ src,
                                                   int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (To)src[i];
}

__global__ void clear_flag_kernel(int32_t *flag) { flag[0] = 0; }

template <typename T>
__global__ __launch_bounds__(256) void nonfinite_kernel(const T *__restrict__ src, int64_t n,
                                                        int32_t *flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(src[i]);
  if (bad) flag[0] = 1;
}

inline int grid_stride_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b < 8192 ? (b < 1 ? 1 : b) : 8192);
}

template <typename T, int DERIV>
hipError_t launch_stage_d(const StageArgs<T> &a, bool ball, hipStream_t s) {
  int64_t blocks = (a.npts + 255) / 256;
  if (ball)
    hipLaunchKernelGGL((stage_generic<T, DERIV, true>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((stage_generic<T, DERIV, false>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_stage(const StageArgs<T> &a, int deriv, bool ball, hipStream_t s) {
  if (deriv == kUpwind1) return launch_stage_d<T, kUpwind1>(a, ball, s);
  return launch_stage_d<T, kEno2>(a, ball, s);
}

template <typename T>
hipError_t launch_cylinders(const CylinderArgs<T> &a, hipStream_t s) {
  hipLaunchKernelGGL(cylinders_kernel<T>, dim3((unsigned)(a.n0 * a.n1)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_alpha_max(const double *ax, const double *ay, int64_t m, double av, double ath,
                            double *alpha_max, hipStream_t s) {
  hipLaunchKernelGGL(alpha_max_kernel, dim3(1), dim3(256), 0, s, ax, ay, m, av, ath, alpha_max);
  return hipGetLastError();
}

template <typename To, typename Ti>
hipError_t launch_cast(To *dst, const Ti *src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((cast_kernel<To, Ti>), dim3(grid_stride_blocks(n)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(T *dst, const T *src, int64_t n, hipStream_t s) {
  return launch_cast<T, T>(dst, src, n, s);
}

template <typename T>
hipError_t launch_nonfinite(const T *src, int64_t n, int32_t *flag, hipStream_t s) {
  hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, s, flag);
  hipLaunchKernelGGL(nonfinite_kernel<T>, dim3(grid_stride_blocks(n)), dim3(256), 0, s, src, n, flag);
  return hipGetLastError();
}

template hipError_t launch_stage<float>(const StageArgs<float> &, int, bool, hipStream_t);
template hipError_t launch_stage<double>(const StageArgs<double> &, int, bool, hipStream_t);
template hipError_t launch_cylinders<float>(const CylinderArgs<float> &, hipStream_t);
template hipError_t launch_cylinders<double>(const CylinderArgs<double> &, hipStream_t);
template hipError_t launch_cast<float, double>(float *, const double *, int64_t, hipStream_t);
template hipError_t launch_cast<double, float>(double *, const float *, int64_t, hipStream_t);
template hipError_t launch_copy<float>(float *, const float *, int64_t, hipStream_t);
template hipError_t launch_copy<double>(double *, const double *, int64_t, hipStream_t);
template hipError_t launch_nonfinite<float>(const float *, int64_t, int32_t *, hipStream_t);
template hipError_t launch_nonfinite<double>(const double *, int64_t, int32_t *, hipStream_t);

}  // namespace hj
