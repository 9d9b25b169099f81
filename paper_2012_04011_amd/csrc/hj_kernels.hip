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

// A block-uniform element of a table that no thread writes during the
// launch, read through the scalar data cache: its latency is then counted
// apart from the vector loads in flight.
template <typename T>
__device__ inline T uniform_load(const T *p, int i) {
  typedef const T __attribute__((address_space(4))) CT;
  return ((CT *)p)[i];
}

// ENO2 works with the undivided second difference at node i in its
// divided-difference form: the first difference on the right minus the one
// on the left, Q_i = (V_{i+1} - V_i) - (V_i - V_{i-1}).  Sweeps that already
// hold the first differences pay one subtraction per Q.

// One-sided derivatives from the window w[0..4] = V_{i-2..i+2} (upwind uses
// w[1..3]).  ENO2: the second-order correction takes the smaller-magnitude
// second difference on the side of the derivative (ties: the left one).
template <typename T, int DERIV>
__device__ inline void one_sided(const T (&w)[5], T inv_h, T &pm, T &pp) {
  if (DERIV == kUpwind1) {
    pm = (w[2] - w[1]) * inv_h;
    pp = (w[3] - w[2]) * inv_h;
  } else {
    T d0 = w[1] - w[0], d1 = w[2] - w[1], d2 = w[3] - w[2], d3 = w[4] - w[3];
    T ql = d1 - d0, qm = d2 - d1, qr = d3 - d2;
    T cm = tabs(ql) <= tabs(qm) ? ql : qm;
    T cp = tabs(qm) <= tabs(qr) ? qm : qr;
    pm = (d1 + T(0.5) * cm) * inv_h;
    pp = (d2 - T(0.5) * cp) * inv_h;
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
__device__ inline T lf_rhs(const T (&pm)[4], const T (&pp)[4], T bx, T by, T ax, T ay, T ath, T sgt,
                           const StageArgs<T> &a) {
  T pb[4], hd[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    pb[d] = T(0.5) * (pp[d] + pm[d]);
    hd[d] = T(0.5) * (pp[d] - pm[d]);
  }
  T L = bx * pb[0] + by * pb[1] + a.bv * pb[2] + a.bth * pb[3];
#pragma unroll
  for (int d = 0; d < 4; ++d) L += (d == 3 ? sgt : a.sig[d]) * tabs(pb[d]);
  L += ax * hd[0] + ay * hd[1] + a.av * hd[2] + ath * hd[3];
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
  if (a.skip && *a.skip) return;
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
  T L = lf_rhs<T, BALL>(pm, pp, bx, by, ax, ay, a.th[idx[2]], a.th[a.n[2] + idx[2]], a);
  a.out[p] = finish(a, p, v[p], L);
}

// ---------------------------------------------------------------------------
// Streaming stage kernel.
//
// Thread r of the grid owns a run of R consecutive theta nodes at one (y, v)
// and sweeps a chunk of x planes in order.  Along x it keeps a register ring
// of the stencil quantities (V_X, V_X+1, the first difference D_X-1/2, the
// second difference Q_X and the ENO choice m_X-1/2), so each new plane costs
// one 16-byte load and one new difference / second difference / choice.
// Along theta the run shares its interface quantities between neighbouring
// nodes (R + 1 first differences and choices for R nodes); the two halo
// nodes on each side are 2-element vector loads (theta wraps).  Along v and y
// the four neighbouring runs are 16-byte loads that the neighbouring threads
// brought into the caches.  Blocks are numbered so that each XCD sweeps one
// contiguous range of runs for one x chunk (their v and y neighbours then sit
// in that XCD's L2), and the pointwise streams (V^n, V0, the output) use
// non-temporal accesses so that they do not push V out of L2.
// ---------------------------------------------------------------------------

template <typename T, int R>
struct VecT {
  typedef T type __attribute__((ext_vector_type(R)));
};
template <typename T>
struct Vec2T {
  typedef T type __attribute__((ext_vector_type(2)));
};
// A run in global memory.  Runs of 3 sit at 12-byte strides and the last
// run of a ragged row starts at any element, so the vector type carries the
// element's alignment only (gfx950 takes 16-byte loads and stores at 4-byte
// alignment; the instructions are the same).
template <typename T, int R>
struct GVecT {
  typedef T type __attribute__((ext_vector_type(R), aligned(sizeof(T))));
};

template <typename T, int R>
__device__ inline void load_run(const T *__restrict__ p, T (&r)[R]) {
  typedef typename GVecT<T, R>::type V;
  V x = *reinterpret_cast<const V *>(p);
#pragma unroll
  for (int i = 0; i < R; ++i) r[i] = x[i];
}

template <typename T, int R>
__device__ inline void load_run_nt(const T *__restrict__ p, T (&r)[R]) {
  typedef typename GVecT<T, R>::type V;
  V x = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
#pragma unroll
  for (int i = 0; i < R; ++i) r[i] = x[i];
}

template <typename T, int R>
__device__ inline void store_run_nt(T *__restrict__ p, const T (&r)[R]) {
  typedef typename GVecT<T, R>::type V;
  V x;
#pragma unroll
  for (int i = 0; i < R; ++i) x[i] = r[i];
  __builtin_nontemporal_store(x, reinterpret_cast<V *>(p));
}

template <typename T>
__device__ inline void load_pair(const T *__restrict__ p, T &a, T &b) {
  typedef typename Vec2T<T>::type V;
  V x = *reinterpret_cast<const V *>(p);
  a = x[0];
  b = x[1];
}

// ENO choice between two second differences: the smaller magnitude, the
// first one on a tie.  m_{k+1/2} = choose(Q_k, Q_{k+1}) is both the
// correction of p+ at node k and of p- at node k+1.
template <typename T>
__device__ inline T choose(T a, T b) {
  return fabs(a) <= fabs(b) ? a : b;
}

// Unscaled one-sided differences (h p-, h p+) from a five-node window.
template <typename T, int DERIV>
__device__ inline void window_diffs(T w0, T w1, T w2, T w3, T w4, T &pm, T &pp) {
  if (DERIV == kUpwind1) {
    pm = w2 - w1;
    pp = w3 - w2;
  } else {
    T d0 = w1 - w0, d1 = w2 - w1, d2 = w3 - w2, d3 = w4 - w3;
    T ql = d1 - d0, qm = d2 - d1, qr = d3 - d2;
    pm = d1 + T(0.5) * choose(ql, qm);
    pp = d2 - T(0.5) * choose(qm, qr);
  }
}

// L_d += kp p+ + km p- + sg |p+ + p-| (+ the axis' share of the ball term).
template <typename T, bool SG, bool BALL>
__device__ inline void accumulate(T &L, T &b2, T kp, T km, T sg, T pp, T pm, bool in_ball, T hih) {
  L = fma(kp, pp, L);
  L = fma(km, pm, L);
  if (SG || BALL) {
    T s = pp + pm;
    if (SG) L = fma(sg, fabs(s), L);
    if (BALL && in_ball) {
      T pb = s * hih;
      b2 = fma(pb, pb, b2);
    }
  }
}

__device__ inline int wrap_or_clamp(int i, int n, bool periodic) {
  if (periodic) return i < 0 ? i + n : (i >= n ? i - n : i);
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// V at x plane xi (any integer within two planes of the grid) for the run at
// in-plane offset off: a load on the grid, a wrapped load on a periodic x,
// else the extrapolated ghost.  xi is uniform over the block.
template <typename T, int R>
__device__ inline void x_plane(const T *__restrict__ v, int xi, int nx, bool periodic, int plane, int off,
                               T (&r)[R]) {
  if (xi >= 0 && xi < nx) {
    load_run<T, R>(v + xi * plane + off, r);
  } else if (periodic) {
    int w = xi < 0 ? xi + nx : xi - nx;
    load_run<T, R>(v + w * plane + off, r);
  } else {
    int e = xi < 0 ? 0 : nx - 1, nb = xi < 0 ? 1 : nx - 2;
    T k = T(xi < 0 ? -xi : xi - (nx - 1));
    T ve[R], vb[R];
    load_run<T, R>(v + e * plane + off, ve);
    load_run<T, R>(v + nb * plane + off, vb);
#pragma unroll
    for (int j = 0; j < R; ++j) r[j] = ve[j] + k * (ve[j] - vb[j]);
  }
}

// Raw buffer access: a 128-bit resource in SGPRs (base, byte range), a
// per-lane byte offset and a wave-uniform byte offset.  Loads past the range
// return zero and stores past it are dropped.
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

constexpr int kCacheDefault = 0;
constexpr int kCacheStream = 2;  // non-temporal

template <typename T, int R, int AUX = kCacheDefault>
__device__ inline void bload(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, T (&r)[R]) {
  typedef typename GVecT<T, R>::type V;
  V x;
  if constexpr (R == 3 && sizeof(T) == 4)
    x = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b96(rs, voff, soff, AUX));
  else if constexpr (sizeof(V) == 16)
    x = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, AUX));
  else if constexpr (sizeof(V) == 8)
    x = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, AUX));
  else
    x = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, AUX));
#pragma unroll
  for (int i = 0; i < R; ++i) r[i] = x[i];
}

template <typename T>
__device__ inline void bload_pair(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, T &a, T &b) {
  typedef typename Vec2T<T>::type V;
  V x;
  if constexpr (sizeof(T) == 4)
    x = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, kCacheDefault));
  else
    x = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, kCacheDefault));
  a = x[0];
  b = x[1];
}

template <typename T>
__device__ inline void bload_one(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, T &a) {
  T r[1];
  bload<T, 1>(rs, voff, soff, r);
  a = r[0];
}

// Element offsets (from `base`, the start of the theta row) of the theta
// halo of the run starting at th0.  R >= 2 (N_theta a multiple of R, so
// even): h[0] = first of the pair (th0-2, th0-1), h[2] = first of the pair
// (th0+R, th0+R+1), each pair contiguous after wrapping.  R = 1: h[k] = the
// wrapped th0-2, th0-1, th0+1, th0+2 (N_theta >= 3).
template <int R>
__device__ inline void theta_halo_offsets(int base, int th0, int nth, uint32_t (&h)[4]) {
  if constexpr (R >= 2) {
    h[0] = (uint32_t)(base + (th0 >= 2 ? th0 - 2 : th0 - 2 + nth));
    h[2] = (uint32_t)(base + (th0 + R < nth ? th0 + R : th0 + R - nth));
    h[1] = h[0] + 1;
    h[3] = h[2] + 1;
  } else {
    const int o[4] = {-2, -1, 1, 2};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int t = th0 + o[k];
      t = t < 0 ? t + nth : (t >= nth ? t - nth : t);
      h[k] = (uint32_t)(base + t);
    }
  }
}

// V at x plane xi (within two planes of the grid) for one run: on the grid,
// wrapped on a periodic x axis, else extrapolated.  xi is block-uniform.
template <typename T, int R>
__device__ inline void x_plane_b(__amdgpu_buffer_rsrc_t rs, int xi, int nx, bool periodic, uint32_t pb, uint32_t voff,
                                 T (&r)[R]) {
  if (xi >= 0 && xi < nx) {
    bload<T, R>(rs, voff, (uint32_t)xi * pb, r);
  } else if (periodic) {
    int w = xi < 0 ? xi + nx : xi - nx;
    bload<T, R>(rs, voff, (uint32_t)w * pb, r);
  } else {
    int e = xi < 0 ? 0 : nx - 1, nb = xi < 0 ? 1 : nx - 2;
    T k = T(xi < 0 ? -xi : xi - (nx - 1));
    T ve[R], vb[R];
    bload<T, R>(rs, voff, (uint32_t)e * pb, ve);
    bload<T, R>(rs, voff, (uint32_t)nb * pb, vb);
#pragma unroll
    for (int j = 0; j < R; ++j) r[j] = ve[j] + k * (ve[j] - vb[j]);
  }
}

// One-sided differences at the nodes next to the ends of an open axis,
// straight from the interior values.  With ghosts extrapolated linearly
// (ghost k layers out = V_end + k (V_end - V_next)), every first difference
// beyond an end equals the last one inside it and the second differences
// there vanish, so the ENO correction on the ghost side is zero and (ENO2
// and upwind alike)
//   i = 0:      h p- = h p+ = V_1 - V_0
//   i = 1:      h p-        = V_1 - V_0
//   i = n - 2:        h p+  = V_{n-1} - V_{n-2}
//   i = n - 1:  h p- = h p+ = V_{n-1} - V_{n-2}.
// This equals the ghost-layer evaluation up to its rounding (a few units in
// the last place of V); the windows of these nodes were loaded with clamped
// indices, and pm, pp computed from them are replaced here.
// An empty volatile asm statement: the compiler may not speculate it, so a
// block holding it stays behind its (wave-uniform) branch instead of being
// turned into selects that every wave executes.
__device__ inline void keep_branch() { asm volatile(""); }

template <typename T>
__device__ inline void edge_diffs(int i, int n, T m1, T c, T p1, T &pm, T &pp) {
  const T dl = c - m1, dr = p1 - c;
  pm = i == 0 ? dr : ((i == 1 || i == n - 1) ? dl : pm);
  pp = i == n - 1 ? dl : ((i == 0 || i == n - 2) ? dr : pp);
}

// One tile of the streaming kernel: logical block lb of the launch that `a`
// describes (blocks_per_chunk run blocks per x chunk, chunk-major).
template <typename T, int R, int DERIV, bool SG, bool BALL>
__device__ inline void stream_tile(const StreamArgs<T> &a, const int lb) {
  constexpr uint32_t E = sizeof(T);
  const int chunk = lb / a.blocks_per_chunk;
  const int r = (lb - chunk * a.blocks_per_chunk) * kStreamBlock + (int)threadIdx.x;
  if (r >= a.slab_runs) return;
  const int nx = a.n[0], ny = a.n[1], nv = a.n[2], nth = a.n[3];
  const bool perx = a.periodic_mask & 1u, pery = (a.periodic_mask >> 1) & 1u, perv = (a.periodic_mask >> 2) & 1u;
  // runs are ordered theta-run fastest, then v, then y: a wave's 64 runs
  // cover one contiguous stretch of a plane
  const int t = r % a.runs_per_row;
  const int yv = r / a.runs_per_row;
  const int v = yv % nv;
  const int y = yv / nv;
  const int th0 = t * R;
  const int rowoff = (y * nv + v) * nth;
  const int offe = rowoff + th0;
  const uint32_t oc = (uint32_t)offe * E;
  // theta halos: two aligned pairs (runs of 2 or 4 on an even N_theta), or
  // four single nodes, each wrapped (runs of 1)
  uint32_t oh[4];
  theta_halo_offsets<R>(rowoff, th0, nth, oh);
  uint32_t ov[4], oy[4];
  {
    const int o[4] = {-2, -1, 1, 2};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      ov[k] = (uint32_t)((y * nv + wrap_or_clamp(v + o[k], nv, perv)) * nth + th0) * E;
      oy[k] = (uint32_t)((wrap_or_clamp(y + o[k], ny, pery) * nv + v) * nth + th0) * E;
    }
  }
  // the edge fix-ups run in the waves that hold an edge lane (branching on a
  // wave-uniform flag keeps the selects out of every other wave)
  const bool vedge = __ballot(!perv && (v < 2 || v >= nv - 2)) != 0;
  const bool yedge = __ballot(!pery && (y < 2 || y >= ny - 2)) != 0;
  // theta-axis coefficients of this thread's v (see StreamArgs::coef_th)
  const T kpt = a.coef_th[v], kmt = a.coef_th[nv + v], sgt = a.coef_th[2 * nv + v];
  T kpx[R], kmx[R], kpy[R], kmy[R];
  {
    const int c = v * nth + th0, m = nv * nth;
    load_run<T, R>(a.coef + c, kpx);
    load_run<T, R>(a.coef + m + c, kmx);
    load_run<T, R>(a.coef + 2 * m + c, kpy);
    load_run<T, R>(a.coef + 3 * m + c, kmy);
  }
  const bool ball_x = (a.ball_mask & 1u) != 0, ball_y = (a.ball_mask & 2u) != 0;
  const bool ball_v = (a.ball_mask & 4u) != 0, ball_t = (a.ball_mask & 8u) != 0;

  const uint32_t pb = (uint32_t)a.plane * E;  // bytes per x plane
  const uint32_t total = pb * (uint32_t)nx;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.vs, total);
  const __amdgpu_buffer_rsrc_t rvn = make_rsrc(a.vn, a.mode == kAverage ? total : 0u);
  const __amdgpu_buffer_rsrc_t rv0 = make_rsrc(a.v0, (a.clamp && !a.v0xy) ? total : 0u);
  const int x0 = chunk * a.chunk_len;
  const int x1 = min(nx, x0 + a.chunk_len);
  constexpr int FR = DERIV == kEno2 ? 2 : 1;  // the x front is plane X + FR

  // x ring (see the description above) and the prefetched front
  T vx0[R], vx1[R], dxm[R], dxp[R], qx0[R], mxm[R], pre[R];
  if (DERIV == kEno2) {
    T wm2[R], wm1[R];
    x_plane_b<T, R>(rs, x0 - 2, nx, perx, pb, oc, wm2);
    x_plane_b<T, R>(rs, x0 - 1, nx, perx, pb, oc, wm1);
    x_plane_b<T, R>(rs, x0, nx, perx, pb, oc, vx0);
    x_plane_b<T, R>(rs, x0 + 1, nx, perx, pb, oc, vx1);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      dxm[j] = vx0[j] - wm1[j];
      dxp[j] = vx1[j] - vx0[j];
      T qm = dxm[j] - (wm1[j] - wm2[j]);
      qx0[j] = dxp[j] - dxm[j];
      mxm[j] = choose(qm, qx0[j]);
    }
  } else {
    T wm1[R];
    x_plane_b<T, R>(rs, x0 - 1, nx, perx, pb, oc, wm1);
    x_plane_b<T, R>(rs, x0, nx, perx, pb, oc, vx0);
#pragma unroll
    for (int j = 0; j < R; ++j) dxm[j] = vx0[j] - wm1[j];
  }
  x_plane_b<T, R>(rs, x0 + FR, nx, perx, pb, oc, pre);
  // y neighbours of the current plane: loaded at the end of the previous
  // plane, as soon as that plane has used them
  T Y[4][R];
  if (DERIV == kEno2) bload<T, R>(rs, oy[0], (uint32_t)x0 * pb, Y[0]);
  bload<T, R>(rs, oy[1], (uint32_t)x0 * pb, Y[1]);
  bload<T, R>(rs, oy[2], (uint32_t)x0 * pb, Y[2]);
  if (DERIV == kEno2) bload<T, R>(rs, oy[3], (uint32_t)x0 * pb, Y[3]);

  for (int X = x0; X < x1; ++X) {
    const uint32_t sX = (uint32_t)X * pb;
    // ---- issue this plane's neighbour loads, then the next front
    T u[R + 4];
    T vn2[R], vn1[R], vp1[R], vp2[R];
    T(&yn2)[R] = Y[0];
    T(&yn1)[R] = Y[1];
    T(&yp1)[R] = Y[2];
    T(&yp2)[R] = Y[3];
    if constexpr (R >= 2) {
      bload_pair<T>(rs, oh[0] * E, sX, u[0], u[1]);
      bload_pair<T>(rs, oh[2] * E, sX, u[R + 2], u[R + 3]);
    } else {
      bload_one<T>(rs, oh[0] * E, sX, u[0]);
      bload_one<T>(rs, oh[1] * E, sX, u[1]);
      bload_one<T>(rs, oh[2] * E, sX, u[3]);
      bload_one<T>(rs, oh[3] * E, sX, u[4]);
    }
    if (DERIV == kEno2) bload<T, R>(rs, ov[0], sX, vn2);
    bload<T, R>(rs, ov[1], sX, vn1);
    bload<T, R>(rs, ov[2], sX, vp1);
    if (DERIV == kEno2) bload<T, R>(rs, ov[3], sX, vp2);
    // pointwise streams of this plane (V^n, V0): issued now, used at the end
    // (the x-y table's value stays one register until the clamp: copying it
    // into t0 here would make the wave wait for every load issued above)
    T vn[R], t0[R], tv = T(0);
    if (a.mode == kAverage) bload<T, R, kCacheStream>(rvn, oc, sX, vn);
    if (a.clamp) {
      // one load feeds tv with either target form (the full-target form
      // reads a value it does not use): no path then overwrites tv while a
      // load into it may be in flight, which would cost a wait for them all
      const T *tp = a.v0xy ? a.v0xy + (X * ny + y) : a.vs;
      tv = *tp;
      if (!a.v0xy) bload<T, R, kCacheStream>(rv0, oc, sX, t0);
    }
    T front[R];
#pragma unroll
    for (int j = 0; j < R; ++j) front[j] = pre[j];
    if (X + 1 < x1) {
      const int xf = X + 1 + FR;
      if (xf < nx)
        bload<T, R>(rs, oc, (uint32_t)xf * pb, pre);
      else
        x_plane_b<T, R>(rs, xf, nx, perx, pb, oc, pre);
    }
    T L[R], b2[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      L[j] = T(0);
      b2[j] = T(0);
    }
    // ---- x: advance the ring; c = V_X (centre)
    T c[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      T pm, pp;
      c[j] = vx0[j];
      if (DERIV == kEno2) {
        T dnn = front[j] - vx1[j];
        T qx1 = dnn - dxp[j];
        T mxp = choose(qx0[j], qx1);
        pm = dxm[j] + T(0.5) * mxm[j];
        pp = dxp[j] - T(0.5) * mxp;
        dxm[j] = dxp[j];
        dxp[j] = dnn;
        qx0[j] = qx1;
        mxm[j] = mxp;
        vx0[j] = vx1[j];
        vx1[j] = front[j];
      } else {
        T dn = front[j] - vx0[j];
        pm = dxm[j];
        pp = dn;
        dxm[j] = dn;
        vx0[j] = front[j];
      }
      accumulate<T, SG, BALL>(L[j], b2[j], kpx[j], kmx[j], a.sg[0], pp, pm, ball_x, a.half_inv_h[0]);
    }
    // ---- theta: the run with its wrapped halos
#pragma unroll
    for (int j = 0; j < R; ++j) u[j + 2] = c[j];
    {
      // e[k] = u[k+1] - u[k]; the second difference at u[k] is e[k] - e[k-1]
      T e[R + 3];
#pragma unroll
      for (int k = 0; k < R + 3; ++k)
        if (DERIV == kEno2 || (k >= 1 && k <= R + 1)) e[k] = u[k + 1] - u[k];  // upwind: no outer halo
      T mprev = T(0);
      if (DERIV == kEno2) mprev = choose(e[1] - e[0], e[2] - e[1]);
#pragma unroll
      for (int j = 0; j < R; ++j) {
        T pm, pp;
        if (DERIV == kEno2) {
          T mnext = choose(e[j + 2] - e[j + 1], e[j + 3] - e[j + 2]);
          pm = e[j + 1] + T(0.5) * mprev;
          pp = e[j + 2] - T(0.5) * mnext;
          mprev = mnext;
        } else {
          pm = e[j + 1];
          pp = e[j + 2];
        }
        accumulate<T, true, BALL>(L[j], b2[j], kpt, kmt, sgt, pp, pm, ball_t, a.half_inv_h[3]);
      }
    }
    // ---- v
    T pmv[R], ppv[R];
#pragma unroll
    for (int j = 0; j < R; ++j) window_diffs<T, DERIV>(vn2[j], vn1[j], c[j], vp1[j], vp2[j], pmv[j], ppv[j]);
    if (vedge) {
      keep_branch();
#pragma unroll
      for (int j = 0; j < R; ++j) edge_diffs<T>(v, nv, vn1[j], c[j], vp1[j], pmv[j], ppv[j]);
    }
#pragma unroll
    for (int j = 0; j < R; ++j)
      accumulate<T, true, BALL>(L[j], b2[j], a.kp_v, a.km_v, a.sg[2], ppv[j], pmv[j], ball_v, a.half_inv_h[2]);
    // ---- y
    T pmy[R], ppy[R];
#pragma unroll
    for (int j = 0; j < R; ++j) window_diffs<T, DERIV>(yn2[j], yn1[j], c[j], yp1[j], yp2[j], pmy[j], ppy[j]);
    if (yedge) {
      keep_branch();
#pragma unroll
      for (int j = 0; j < R; ++j) edge_diffs<T>(y, ny, yn1[j], c[j], yp1[j], pmy[j], ppy[j]);
    }
#pragma unroll
    for (int j = 0; j < R; ++j)
      accumulate<T, SG, BALL>(L[j], b2[j], kpy[j], kmy[j], a.sg[1], ppy[j], pmy[j], ball_y, a.half_inv_h[1]);
    if (X + 1 < x1) {
      if (DERIV == kEno2) bload<T, R>(rs, oy[0], sX + pb, Y[0]);
      bload<T, R>(rs, oy[1], sX + pb, Y[1]);
      bload<T, R>(rs, oy[2], sX + pb, Y[2]);
      if (DERIV == kEno2) bload<T, R>(rs, oy[3], sX + pb, Y[3]);
    }
    // ---- update
    T res[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      T Lj = L[j];
      if (BALL) Lj = fma(a.sig_ball, sqrt(b2[j]), Lj);
      res[j] = fma(a.dt, Lj, c[j]);
    }
    if (a.mode == kAverage) {
#pragma unroll
      for (int j = 0; j < R; ++j) res[j] = T(0.5) * (vn[j] + res[j]);
    }
    if (a.clamp) {
      if (a.v0xy) {
#pragma unroll
        for (int j = 0; j < R; ++j) res[j] = tv < res[j] ? tv : res[j];
      } else {
#pragma unroll
        for (int j = 0; j < R; ++j) res[j] = t0[j] < res[j] ? t0[j] : res[j];
      }
    }
    // a global (not buffer) store: with a register soffset the compiler puts
    // no wait state between a 128-bit buffer store and the next write of its
    // data registers, and outputs came out wrong at random under load
    store_run_nt<T, R>(a.out + (size_t)X * a.plane + offe, res);
  }
}

template <typename T, int R, int DERIV, bool SG, bool BALL>
__global__ __launch_bounds__(kStreamBlock) void stage_stream(StreamArgs<T> a) {
  if (a.skip && *a.skip) return;
  stream_tile<T, R, DERIV, SG, BALL>(a, (int)xcd_logical_block(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// Plane kernel.  Block (y, x chunk) owns every run of the (v, theta) plane at
// one y (or of one v segment of it, see SEG) and sweeps the chunk's x
// planes.  Each thread keeps the x ring of its run in registers; per plane it
// writes its centre run into a double-buffered LDS copy of the plane, and
// after one barrier reads its theta halos and its v neighbours from LDS.
// Only the x front (prefetched one plane ahead), the four y-neighbour runs
// and the pointwise streams (V^n, V0) are global loads.
// ---------------------------------------------------------------------------

template <typename T, int R>
__device__ inline void lds_run(const T *p, T (&r)[R]) {
  // a run of 3 sits in a 4-element slot (16-byte aligned)
  typedef typename VecT<T, R == 3 ? 4 : R>::type V;
  V x = *reinterpret_cast<const V *>(p);
#pragma unroll
  for (int i = 0; i < R; ++i) r[i] = x[i];
}

template <typename T>
__device__ inline void lds_pair(const T *p, T &a, T &b) {
  typedef typename Vec2T<T>::type V;
  V x = *reinterpret_cast<const V *>(p);
  a = x[0];
  b = x[1];
}

__device__ inline double wave_max_d(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double y = __shfl_xor(x, o, 64);
    x = y > x ? y : x;
  }
  return x;
}

__device__ inline unsigned long long order_key(double x) {
  unsigned long long b = (unsigned long long)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// Stage forms the plane kernel compiles in (see FORM below): Euler or TVD-RK2
// stage 1 without a clamp, the last stage of an Euler step with the clamp
// value from the Nx x Ny table, TVD-RK2 stage 2 (the average) with it, and
// that stage folding eps = max |V^n+1 - V^n| (convergence mode; a.eps set).
enum PlaneForm { kFormRuntime = 0, kFormPlain = 1, kFormPlainXY = 2, kFormAverageXY = 3, kFormAverageXYEps = 4 };

// SEG: the block holds one v segment [va, va + v_seg) of the plane plus two
// halo rows on each side (copied from global memory by the first 4 * rpr
// threads, one plane ahead), for planes with more runs than a block has
// threads.
// FORM: the stage's combine and clamp target fixed at compile time for the
// forms the solves use (PlaneForm), so that every plane issues the same
// memory operations and branches on none of them; kFormRuntime reads them,
// and the eps fold, from the arguments.
// R = 3 (FP32): runs of three theta nodes, each kept in a 4-element LDS slot
// (16-byte aligned), blocks of up to kPlaneMaxThreads3 work-items.
// One block of the plane kernel: logical block lb of the nblk blocks of the
// grid's launch (a single-grid launch, or the grid's share of a batched one).
// ROWS2 (chunk mode): the block holds two neighbouring y rows, y0 = 2u and
// y0 + 1, of one v segment (or of the whole plane); the threads of row q
// start at q * tpr, a whole number of waves.  Along y each thread loads only
// its two outer neighbours from memory -- y0 - 2 and y0 - 1 for row 0,
// y0 + 2 and y0 + 3 for row 1 -- two planes ahead.  The inner ones come from
// LDS: the other row's centre (its plane buffer) and the neighbour the other
// row loaded (row 0 publishes y0 - 1, row 1 publishes y0 + 2).  Every node
// sees the values of the one-row block, so the results are the same.
template <typename T, int R, int DERIV, bool SG, bool BALL, bool SEG, bool RANGE, int FORM, bool ROWS2 = false>
__device__ __forceinline__ void plane_block(const StreamArgs<T> &a, const int lb, const int nblk) {
  static_assert(!(ROWS2 && RANGE), "two-row blocks run the stage only");
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T *lds = reinterpret_cast<T *>(lds_raw);
  constexpr uint32_t E = sizeof(T);
  const int nx = a.n[0], ny = a.n[1], nv = a.n[2], nth = a.n[3];
  const int rpr = a.runs_per_row;
  constexpr int SL = R == 3 ? 4 : R;  // LDS elements per run
  const int rowl = rpr * SL;          // LDS elements per v row
  // ROWS2: threads per row (whole waves) and this thread's row, uniform over
  // the wave
  const int tpr = ROWS2 ? ((SEG ? a.v_seg : nv) * rpr + 63) / 64 * 64 : 0;
  const int row2 = ROWS2 ? (int)__builtin_amdgcn_readfirstlane((int)threadIdx.x >= tpr ? 1 : 0) : 0;
  const int tl = (int)threadIdx.x - row2 * tpr;  // the thread's index inside its row
  const int nyu = ROWS2 ? ny / 2 : ny;            // y units (rows, or row pairs) per segment
  // chunk mode (a.span == 0): the block is (x chunk, v segment, y unit).
  // Span mode (whole planes, SEG false): the block takes its equal share of
  // all rows' x planes in row-major order, as one or more (row, x range)
  // segments; gridDim.x blocks share the ny * nx row-planes.
  const int chunk = a.span ? 0 : lb / a.blocks_per_chunk;
  const int rem = a.span ? 0 : lb - chunk * a.blocks_per_chunk;  // segment-major, y fastest
  const int seg = SEG ? rem / nyu : 0;
  const int va = seg * a.v_seg;                            // first v of the segment
  const int nvs = SEG ? min(a.v_seg, nv - va) : nv;        // its rows
  const int vbase = SEG ? va - 2 : 0;                      // v of LDS row 0
  const int runs = nvs * rpr;                              // runs of the block (of each row)
  const bool active = tl < runs;
  const int r = active ? tl : runs - 1;  // idle lanes shadow the last run
  const bool perx = a.periodic_mask & 1u, pery = (a.periodic_mask >> 1) & 1u, perv = (a.periodic_mask >> 2) & 1u;
  const int t = r % rpr;
  const int v = va + r / rpr;
  // ragged rows (runs of 2 or 4 that do not divide N_theta, whole planes):
  // the last run of a row starts at N_theta - R, repeating the last nodes of
  // the run before it (both compute them alike and store the same values)
  const bool ragged = !SEG && (R == 2 || R == 4) && rpr * R != nth;  // whole planes only
  const int th0 = (ragged && t == rpr - 1) ? nth - R : t * R;
  const int pl = v * nth + th0;             // offset inside the (v, theta) plane
  const int pll = (v - vbase) * rowl + t * SL;  // the run's slot in the LDS copy
  int lv[4];
  {
    const int o[4] = {-2, -1, 1, 2};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      // a segment's halo rows hold v - 2 .. v + 2 unwrapped on a periodic v
      const int vk = (SEG && perv) ? v + o[k] : wrap_or_clamp(v + o[k], nv, perv);
      lv[k] = (vk - vbase) * rowl + t * SL;
    }
  }
  uint32_t lh[4];  // theta halos inside the LDS plane (see the streaming kernel)
  if constexpr (R == 3) {
    // the last two elements of the previous run's slot, the first two of the next run's
    const int base = (v - vbase) * rowl;
    lh[0] = (uint32_t)(base + (t == 0 ? rpr - 1 : t - 1) * SL + 1);
    lh[1] = lh[0] + 1;
    lh[2] = (uint32_t)(base + (t == rpr - 1 ? 0 : t + 1) * SL);
    lh[3] = lh[2] + 1;
  } else if (ragged) {
    // the LDS row holds theta 0 .. (rpr - 1) R - 1 in place and the last
    // run's R nodes after them
    const int base = (v - vbase) * rowl, lim = (rpr - 1) * R, shift = rpr * R - nth;
    const int o[4] = {-2, -1, R, R + 1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int q = th0 + o[k];
      q = q < 0 ? q + nth : (q >= nth ? q - nth : q);
      lh[k] = (uint32_t)(base + (q < lim ? q : q + shift));
    }
  } else {
    theta_halo_offsets<R>((v - vbase) * nth, th0, nth, lh);
  }
  // the v fix-ups run in the waves that hold an edge lane (branching on a
  // wave-uniform flag keeps the selects out of every other wave); y is the
  // block's
  const bool vedge = __ballot(!perv && (v < 2 || v >= nv - 2)) != 0;
  // theta-axis coefficients of this thread's v (see StreamArgs::coef_th)
  const T kpt = a.coef_th[v], kmt = a.coef_th[nv + v], sgt = a.coef_th[2 * nv + v];
  T kpx[R], kmx[R], kpy[R], kmy[R];
  {
    const int m = nv * nth;
    load_run<T, R>(a.coef + pl, kpx);
    load_run<T, R>(a.coef + m + pl, kmx);
    load_run<T, R>(a.coef + 2 * m + pl, kpy);
    load_run<T, R>(a.coef + 3 * m + pl, kmy);
  }
  const bool ball_x = (a.ball_mask & 1u) != 0, ball_y = (a.ball_mask & 2u) != 0;
  const bool ball_v = (a.ball_mask & 4u) != 0, ball_t = (a.ball_mask & 8u) != 0;
  // the stage's form: compile-time constants unless FORM is kFormRuntime
  constexpr bool kRT = FORM == kFormRuntime;
  const bool avg = kRT ? a.mode == kAverage : (FORM == kFormAverageXY || FORM == kFormAverageXYEps);
  const bool clamp = kRT ? a.clamp != 0 : FORM != kFormPlain;
  const bool xy = kRT ? a.v0xy != nullptr : true;  // clamp value from the Nx x Ny table
  const bool fold_eps = kRT ? a.eps != nullptr : FORM == kFormAverageXYEps;

  const uint32_t pb = (uint32_t)a.plane * E;
  const uint32_t total = pb * (uint32_t)nx;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.vs, total);
  const __amdgpu_buffer_rsrc_t rnull = make_rsrc(a.vs, 0u);  // loads through it return 0, no memory access
  const __amdgpu_buffer_rsrc_t rvn = make_rsrc(a.vn, avg ? total : 0u);
  const __amdgpu_buffer_rsrc_t rv0 = make_rsrc(a.v0, (clamp && !xy) ? total : 0u);
  constexpr int FR = DERIV == kEno2 ? 2 : 1;
  const int psz = (SEG ? a.v_seg + 4 : nv) * rowl;  // values per LDS buffer
  // ROWS2: after the four plane buffers (row 0, row 1; two phases each), four
  // buffers of the published y neighbours, and this run's slot in them
  const int xsz = ROWS2 ? (SEG ? a.v_seg : nv) * rowl : 0;
  const int xsl = ROWS2 ? (v - va) * rowl + t * SL : 0;

  // the accumulators of the range pass and the eps fold span every segment
  // RANGE: the smallest and largest derivative (unscaled, h p) per axis
  // over this thread's nodes -- of the central one (p- + p+) / 2, or of both
  // one-sided ones; nothing is written but the keys
  T rlo[4], rhi[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    rlo[d] = T(INFINITY);
    rhi[d] = T(-INFINITY);
  }
  const bool onesided = a.range_onesided != 0;
  auto rng = [&](int d, T pm, T pp) {
    if (!active) return;
    const T cen = T(0.5) * (pm + pp);
    const T mn = onesided ? (pm < pp ? pm : pp) : cen, mx = onesided ? (pm < pp ? pp : pm) : cen;
    rlo[d] = mn < rlo[d] ? mn : rlo[d];
    rhi[d] = mx > rhi[d] ? mx : rhi[d];
  };
  double em = 0.0;  // largest change of this thread's nodes (when a.eps is set)
  int pcb = 0;  // planes done in earlier segments (the LDS buffer's parity)
  int64_t idx = 0, idx_end = 1;  // span mode: this block's row-planes
  if (a.span) {
    const int64_t W = (int64_t)ny * nx;
    idx = (int64_t)lb * W / nblk;
    idx_end = ((int64_t)lb + 1) * W / nblk;
  }
  while (idx < idx_end) {
    // this segment: row y, planes [x0, x1)
    const int yu = SEG ? rem - seg * nyu : rem;
    const int y = a.span ? (int)(idx / nx) : (ROWS2 ? 2 * yu + row2 : yu);
    const int x0 = a.span ? (int)(idx - (int64_t)y * nx) : chunk * a.chunk_len;
    const int x1 = a.span ? (int)min((int64_t)nx, x0 + (idx_end - idx)) : min(nx, x0 + a.chunk_len);
    idx = a.span ? idx + (x1 - x0) : idx_end;
    const int offe = y * nv * nth + pl;
    const uint32_t oc = (uint32_t)offe * E;
    uint32_t oy[4];
    {
      const int o[4] = {-2, -1, 1, 2};
  #pragma unroll
      for (int k = 0; k < 4; ++k) oy[k] = (uint32_t)((wrap_or_clamp(y + o[k], ny, pery) * nv + v) * nth + th0) * E;
    }
    // ROWS2: the neighbours this thread loads (ENO2: y - 2, y - 1 in row 0,
    // y + 1, y + 2 in row 1; first order: y - 1, y + 1)
    const uint32_t og0 = DERIV == kEno2 ? (row2 == 0 ? oy[0] : oy[2]) : (row2 == 0 ? oy[1] : oy[2]);
    const uint32_t og1 = row2 == 0 ? oy[1] : oy[3];
    const bool yedge = !pery && (y < 2 || y >= ny - 2);
    // SEG halo rows va-2, va-1, va+nvs, va+nvs+1 (those that exist): thread
    // h < 4 rpr copies run h % rpr of row h / rpr, loading it one plane ahead
    bool hcopy = false;
    uint32_t hoff = 0;
    int hl = 0;
    T H[R];
    if constexpr (SEG) {
      const int h = tl, hk = h / rpr, ht = h - hk * rpr;
      const int hv = hk < 2 ? va - 2 + hk : va + nvs + (hk - 2);
      hcopy = h < 4 * rpr && (perv || (hv >= 0 && hv < nv));
      const int hw = hv < 0 ? hv + nv : (hv >= nv ? hv - nv : hv);
      // every lane issues the load, so that each plane issues a fixed set of
      // loads; the lanes that copy nothing load at the end of the buffer
      // (lane offset total), out of range: 0 without a memory access (their
      // H is never used)
      hoff = hcopy ? (uint32_t)((y * nv + hw) * nth + ht * R) * E : total;
      hl = (hv - vbase) * rowl + ht * SL;
      bload<T, R>(rs, hoff, (uint32_t)x0 * pb, H);
    }

    // x ring: slot S[(P + k) & 3] holds V(X + k) at phase P = (X - x0) & 3
    // (k = 0 .. FR, and the front of the next plane loading into the last);
    // the rotating slots and the difference pairs need no register moves once
    // the loop is unrolled by four.  D[(P + k) & 3] = V(X + k) - V(X + k - 1)
    // for k = 0, 1 (and 2 once computed); Q[i], M[i]: the second difference at
    // X and the ENO choice between X-1 and X, for the current (i = P & 1) and
    // next plane.
    T S[4][R], D[4][R], Q[2][R], M[2][R];
    if (DERIV == kEno2) {
      T wm2[R], wm1[R];
      x_plane_b<T, R>(rs, x0 - 2, nx, perx, pb, oc, wm2);
      x_plane_b<T, R>(rs, x0 - 1, nx, perx, pb, oc, wm1);
      x_plane_b<T, R>(rs, x0, nx, perx, pb, oc, S[0]);
      x_plane_b<T, R>(rs, x0 + 1, nx, perx, pb, oc, S[1]);
  #pragma unroll
      for (int j = 0; j < R; ++j) {
        D[0][j] = S[0][j] - wm1[j];
        D[1][j] = S[1][j] - S[0][j];
        T qm = D[0][j] - (wm1[j] - wm2[j]);
        Q[0][j] = D[1][j] - D[0][j];
        M[0][j] = choose(qm, Q[0][j]);
      }
    } else {
      T wm1[R];
      x_plane_b<T, R>(rs, x0 - 1, nx, perx, pb, oc, wm1);
      x_plane_b<T, R>(rs, x0, nx, perx, pb, oc, S[0]);
  #pragma unroll
      for (int j = 0; j < R; ++j) D[0][j] = S[0][j] - wm1[j];
    }
    x_plane_b<T, R>(rs, x0 + FR, nx, perx, pb, oc, S[FR]);
    // y neighbours of the current plane (y - 2, y - 1, y + 1, y + 2): loaded
    // at the end of the previous plane, as soon as that plane has used them
    T Y[4][R];
    // ROWS2: this thread's y neighbours of planes x0 and x0 + 1, slot
    // (X - x0) & 1; each plane loads those of X + 2 into its own slot
    T YG[2][2][R];
    if constexpr (ROWS2) {
      const bool on1 = x0 + 1 < x1;
      bload<T, R>(rs, og0, (uint32_t)x0 * pb, YG[0][0]);
      if (DERIV == kEno2) bload<T, R>(rs, og1, (uint32_t)x0 * pb, YG[0][1]);
      bload<T, R>(on1 ? rs : rnull, og0, on1 ? (uint32_t)(x0 + 1) * pb : 0u, YG[1][0]);
      if (DERIV == kEno2) bload<T, R>(on1 ? rs : rnull, og1, on1 ? (uint32_t)(x0 + 1) * pb : 0u, YG[1][1]);
    } else {
      if (DERIV == kEno2) bload<T, R>(rs, oy[0], (uint32_t)x0 * pb, Y[0]);
      bload<T, R>(rs, oy[1], (uint32_t)x0 * pb, Y[1]);
      bload<T, R>(rs, oy[2], (uint32_t)x0 * pb, Y[2]);
      if (DERIV == kEno2) bload<T, R>(rs, oy[3], (uint32_t)x0 * pb, Y[3]);
    }
    auto plane = [&](auto phase, const int X) {
      constexpr int P = decltype(phase)::value;
      constexpr int I0 = P & 3, I1 = (P + 1) & 3, IF = (P + FR) & 3, IL = (P + FR + 1) & 3;
      constexpr int DC = P & 1, DN = (P + 1) & 1;
      const uint32_t sX = (uint32_t)X * pb;
      // LDS planes alternate across segments too; ROWS2: this row's pair of
      // buffers, the other row's beside it
      const int par = (pcb + P) & 1;
      T *buf = lds + (row2 * 2 + par) * psz;
      // ---- the front of this plane (V(X + FR), loaded by the previous plane)
      // lies beyond the end of an open x axis: its ghost, k layers out, from the
      // two end planes in the ring (the slot of V(X - 1) is still unwritten)
      if (X > x0 && !perx && X + FR >= nx) {
        const int k = X + FR - (nx - 1);
        if (k == 1) {
  #pragma unroll
          for (int j = 0; j < R; ++j)
            S[IF][j] = S[(P + FR - 1) & 3][j] + T(1) * (S[(P + FR - 1) & 3][j] - S[(P + FR - 2) & 3][j]);
        } else {
  #pragma unroll
          for (int j = 0; j < R; ++j)
            S[IF][j] = S[(P + FR - 2) & 3][j] + T(2) * (S[(P + FR - 2) & 3][j] - S[(P + FR - 3) & 3][j]);
        }
      }
      // ---- global loads of this plane (its y neighbours are in flight), then the next front
      T(&yn2)[R] = Y[0];
      T(&yn1)[R] = Y[1];
      T(&yp1)[R] = Y[2];
      T(&yp2)[R] = Y[3];
      // pointwise streams of this plane (V^n, V0): issued now, used at the end
      T vn[R], t0[R], tv = T(0);
      if (avg) bload<T, R, kCacheStream>(rvn, oc, sX, vn);
      if (clamp) {
        if (xy)
          tv = uniform_load(a.v0xy, X * ny + y);  // every run of the block shares (x, y)
        else
          bload<T, R, kCacheStream>(rv0, oc, sX, t0);
      }
      {
        // the next front, one load on every plane: none on the chunk's last
        // plane and none beyond the end of an open x (its ghost is formed at
        // the top of the plane that uses it) -- both through the empty
        // resource; a periodic x wraps
        const int xf = X + 1 + FR;
        const bool on = X + 1 < x1 && (perx || xf < nx);
        bload<T, R>(on ? rs : rnull, oc, on ? (uint32_t)(xf < nx ? xf : xf - nx) * pb : 0u, S[IL]);
      }
      // ---- publish the centre run; c = V_X
      const T(&c)[R] = S[I0];
      if (active) {
        typedef typename VecT<T, SL>::type V;
        V cv;
  #pragma unroll
        for (int j = 0; j < SL; ++j) cv[j] = j < R ? c[j] : T(0);
        *reinterpret_cast<V *>(buf + pll) = cv;
        if constexpr (ROWS2 && DERIV == kEno2) {
          // the outer neighbour the other row needs: y0 - 1 (row 0), y0 + 2 (row 1)
          V xv;
  #pragma unroll
          for (int j = 0; j < SL; ++j) xv[j] = j < R ? (row2 == 0 ? YG[P & 1][1][j] : YG[P & 1][0][j]) : T(0);
          *reinterpret_cast<V *>(lds + 4 * psz + (row2 * 2 + par) * xsz + xsl) = xv;
        }
      }
      if constexpr (SEG) {
        if (hcopy) {
          typedef typename VecT<T, R>::type V;
          V hv;
  #pragma unroll
          for (int j = 0; j < R; ++j) hv[j] = H[j];
          *reinterpret_cast<V *>(buf + hl) = hv;
        }
        bload<T, R>(X + 1 < x1 ? rs : rnull, hoff, X + 1 < x1 ? sX + pb : 0u, H);
      }
      T L[R], b2[R];
  #pragma unroll
      for (int j = 0; j < R; ++j) {
        L[j] = T(0);
        b2[j] = T(0);
      }
      // ---- x from the ring (registers only, overlaps the barrier wait)
  #pragma unroll
      for (int j = 0; j < R; ++j) {
        T pm, pp;
        if (DERIV == kEno2) {
          D[(P + 2) & 3][j] = S[IF][j] - S[I1][j];
          Q[DN][j] = D[(P + 2) & 3][j] - D[(P + 1) & 3][j];
          M[DN][j] = choose(Q[DC][j], Q[DN][j]);
          pm = D[P & 3][j] + T(0.5) * M[DC][j];
          pp = D[(P + 1) & 3][j] - T(0.5) * M[DN][j];
        } else {
          D[(P + 1) & 3][j] = S[IF][j] - S[I0][j];
          pm = D[P & 3][j];
          pp = D[(P + 1) & 3][j];
        }
        if constexpr (RANGE)
          rng(0, pm, pp);
        else
          accumulate<T, SG, BALL>(L[j], b2[j], kpx[j], kmx[j], a.sg[0], pp, pm, ball_x, a.half_inv_h[0]);
      }
      __syncthreads();
      // ---- theta: halos from LDS
      {
        T u[R + 4];
        if constexpr (R == 3) {
          u[0] = buf[lh[0]];  // a 4-byte aligned pair
          u[1] = buf[lh[1]];
          lds_pair<T>(buf + lh[2], u[R + 2], u[R + 3]);
        } else if constexpr (R >= 2) {
          if (ragged) {  // the halo pairs may straddle the last run's slot
            u[0] = buf[lh[0]];
            u[1] = buf[lh[1]];
            u[R + 2] = buf[lh[2]];
            u[R + 3] = buf[lh[3]];
          } else {
            lds_pair<T>(buf + lh[0], u[0], u[1]);
            lds_pair<T>(buf + lh[2], u[R + 2], u[R + 3]);
          }
        } else {
          u[0] = buf[lh[0]];
          u[1] = buf[lh[1]];
          u[3] = buf[lh[2]];
          u[4] = buf[lh[3]];
        }
  #pragma unroll
        for (int j = 0; j < R; ++j) u[j + 2] = c[j];
        // e[k] = u[k+1] - u[k]; the second difference at u[k] is e[k] - e[k-1]
        T e[R + 3];
  #pragma unroll
        for (int k = 0; k < R + 3; ++k)
          if (DERIV == kEno2 || (k >= 1 && k <= R + 1)) e[k] = u[k + 1] - u[k];  // upwind: no outer halo
        T mprev = T(0);
        if (DERIV == kEno2) mprev = choose(e[1] - e[0], e[2] - e[1]);
  #pragma unroll
        for (int j = 0; j < R; ++j) {
          T pm, pp;
          if (DERIV == kEno2) {
            T mnext = choose(e[j + 2] - e[j + 1], e[j + 3] - e[j + 2]);
            pm = e[j + 1] + T(0.5) * mprev;
            pp = e[j + 2] - T(0.5) * mnext;
            mprev = mnext;
          } else {
            pm = e[j + 1];
            pp = e[j + 2];
          }
          if constexpr (RANGE)
            rng(3, pm, pp);
          else
            accumulate<T, true, BALL>(L[j], b2[j], kpt, kmt, sgt, pp, pm, ball_t, a.half_inv_h[3]);
        }
      }
      // ---- v: neighbours from LDS
      {
        T vn2[R], vn1[R], vp1[R], vp2[R];
        if (DERIV == kEno2) lds_run<T, R>(buf + lv[0], vn2);
        lds_run<T, R>(buf + lv[1], vn1);
        lds_run<T, R>(buf + lv[2], vp1);
        if (DERIV == kEno2) lds_run<T, R>(buf + lv[3], vp2);
        T pmv[R], ppv[R];
  #pragma unroll
        for (int j = 0; j < R; ++j) window_diffs<T, DERIV>(vn2[j], vn1[j], c[j], vp1[j], vp2[j], pmv[j], ppv[j]);
        if (vedge) {
          keep_branch();
  #pragma unroll
          for (int j = 0; j < R; ++j) edge_diffs<T>(v, nv, vn1[j], c[j], vp1[j], pmv[j], ppv[j]);
        }
  #pragma unroll
        for (int j = 0; j < R; ++j) {
          if constexpr (RANGE)
            rng(2, pmv[j], ppv[j]);
          else
            accumulate<T, true, BALL>(L[j], b2[j], a.kp_v, a.km_v, a.sg[2], ppv[j], pmv[j], ball_v, a.half_inv_h[2]);
        }
      }
      // ---- y: neighbours from global memory (ROWS2: the inner ones from LDS)
      T pmy[R], ppy[R];
      auto ywin = [&](const T(&w0)[R], const T(&w1)[R], const T(&w3)[R], const T(&w4)[R]) {
  #pragma unroll
        for (int j = 0; j < R; ++j) window_diffs<T, DERIV>(w0[j], w1[j], c[j], w3[j], w4[j], pmy[j], ppy[j]);
        if (yedge) {
          keep_branch();
  #pragma unroll
          for (int j = 0; j < R; ++j) edge_diffs<T>(y, ny, w1[j], c[j], w3[j], pmy[j], ppy[j]);
        }
      };
      if constexpr (ROWS2) {
        // the other row's centre, and (ENO2) the neighbour it published
        T oc2[R], ox2[R];
        lds_run<T, R>(lds + ((1 - row2) * 2 + par) * psz + pll, oc2);
        if (DERIV == kEno2) lds_run<T, R>(lds + 4 * psz + ((1 - row2) * 2 + par) * xsz + xsl, ox2);
        const T(&g0)[R] = YG[P & 1][0];
        const T(&g1)[R] = YG[P & 1][1];
        if (row2 == 0) {  // uniform over the wave
          keep_branch();
          if (DERIV == kEno2)
            ywin(g0, g1, oc2, ox2);  // y - 2, y - 1 | y + 1, y + 2
          else
            ywin(g0, g0, oc2, oc2);  // y - 1 | y + 1
        } else {
          keep_branch();
          if (DERIV == kEno2)
            ywin(ox2, oc2, g0, g1);
          else
            ywin(oc2, oc2, g0, g0);
        }
      } else {
        ywin(yn2, yn1, yp1, yp2);
      }
  #pragma unroll
      for (int j = 0; j < R; ++j) {
        if constexpr (RANGE)
          rng(1, pmy[j], ppy[j]);
        else
          accumulate<T, SG, BALL>(L[j], b2[j], kpy[j], kmy[j], a.sg[1], ppy[j], pmy[j], ball_y, a.half_inv_h[1]);
      }
      if constexpr (ROWS2) {
        // this thread's y neighbours of plane X + 2 (none beyond the chunk)
        const bool on2 = X + 2 < x1;
        const __amdgpu_buffer_rsrc_t ry = on2 ? rs : rnull;
        const uint32_t s2 = on2 ? sX + 2 * pb : 0u;
        bload<T, R>(ry, og0, s2, YG[P & 1][0]);
        if (DERIV == kEno2) bload<T, R>(ry, og1, s2, YG[P & 1][1]);
      } else {
        // the next plane's y neighbours (none after the chunk's last plane)
        const __amdgpu_buffer_rsrc_t ry = X + 1 < x1 ? rs : rnull;
        if (DERIV == kEno2) bload<T, R>(ry, oy[0], sX + pb, Y[0]);
        bload<T, R>(ry, oy[1], sX + pb, Y[1]);
        bload<T, R>(ry, oy[2], sX + pb, Y[2]);
        if (DERIV == kEno2) bload<T, R>(ry, oy[3], sX + pb, Y[3]);
      }
      if constexpr (!RANGE) {
        // ---- update
        T res[R];
    #pragma unroll
        for (int j = 0; j < R; ++j) {
          T Lj = L[j];
          if (BALL) Lj = fma(a.sig_ball, sqrt(b2[j]), Lj);
          res[j] = fma(a.dt, Lj, c[j]);
        }
        if (avg) {
    #pragma unroll
          for (int j = 0; j < R; ++j) res[j] = T(0.5) * (vn[j] + res[j]);
        }
        if (clamp) {
          if (xy) {
    #pragma unroll
            for (int j = 0; j < R; ++j) res[j] = tv < res[j] ? tv : res[j];
          } else {
    #pragma unroll
            for (int j = 0; j < R; ++j) res[j] = t0[j] < res[j] ? t0[j] : res[j];
          }
        }
        if (fold_eps) {
    #pragma unroll
          for (int j = 0; j < R; ++j) {
            double d = fabs((double)res[j] - (double)(avg ? vn[j] : c[j]));
            if (d != d) d = INFINITY;
            em = (active && d > em) ? d : em;
          }
        }
        // idle lanes shadow the last run and would store the same values to
        // the same address: in FP32 the store takes no branch (measured
        // faster), in FP64 it keeps it (measured faster that way)
        if (sizeof(T) == 4 || active) store_run_nt<T, R>(a.out + (size_t)X * a.plane + offe, res);
      }
    };

    // four planes per trip: every slot index above is a compile-time constant
    int X = x0;
    for (;;) {
      if (X >= x1) break;
      plane(std::integral_constant<int, 0>(), X++);
      if (X >= x1) break;
      plane(std::integral_constant<int, 1>(), X++);
      if (X >= x1) break;
      plane(std::integral_constant<int, 2>(), X++);
      if (X >= x1) break;
      plane(std::integral_constant<int, 3>(), X++);
    }

    pcb += x1 - x0;
  }
  if (fold_eps) {
    em = wave_max_d(em);
    if ((threadIdx.x & 63) == 0) atomicMax(a.eps, (unsigned long long)__double_as_longlong(em));
  }
  if constexpr (RANGE) {
    // p = (h p) / h; the scaling is monotone, so the extremes scale as they
    // are.  Keys per wave into one of kRangeSlots sets.
    unsigned long long *set = a.range + 8 * ((blockIdx.x * 16 + (threadIdx.x >> 6)) % kRangeSlots);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const T ih = T(2) * a.half_inv_h[d];
      unsigned long long kl = order_key((double)(rlo[d] * ih)), kh = order_key((double)(rhi[d] * ih));
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long ol = __shfl_xor(kl, o, 64), oh = __shfl_xor(kh, o, 64);
        kl = ol < kl ? ol : kl;
        kh = oh > kh ? oh : kh;
      }
      if ((threadIdx.x & 63) == 0) {
        atomicMin(&set[d], kl);
        atomicMax(&set[4 + d], kh);
      }
    }
  }
}

template <typename T, int R, int DERIV, bool SG, bool BALL, bool SEG, bool RANGE, int FORM, bool ROWS2 = false>
__global__ __launch_bounds__(R == 3 ? kPlaneMaxThreads3 : kPlaneMaxThreads) void stage_plane(StreamArgs<T> a) {
  if (a.skip && *a.skip) return;  // uniform over the block: no barrier is skipped by part of it
  plane_block<T, R, DERIV, SG, BALL, SEG, RANGE, FORM, ROWS2>(a, (int)xcd_logical_block(blockIdx.x, gridDim.x),
                                                              (int)gridDim.x);
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
  if (a.combine) {
    T old = a.v0xy[ij];
    best = old < best ? old : best;
  }
  int64_t base = (int64_t)ij * a.plane;
  for (int64_t q = threadIdx.x; q < a.plane; q += blockDim.x) {
    a.v0[base + q] = best;
    if (a.v) a.v[base + q] = best;
  }
  if (threadIdx.x == 0) a.v0xy[ij] = best;
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

template <typename T, int R, int DERIV, bool SG, bool BALL>
hipError_t launch_stream_r(const StreamArgs<T> &a, hipStream_t s) {
  unsigned blocks = (unsigned)(a.blocks_per_chunk * a.n_chunks);
  hipLaunchKernelGGL((stage_stream<T, R, DERIV, SG, BALL>), dim3(blocks), dim3(kStreamBlock), 0, s, a);
  return hipGetLastError();
}

template <typename T, int DERIV, bool SG, bool BALL>
hipError_t launch_stream_v(const StreamArgs<T> &a, hipStream_t s) {
  if (a.run == 1) return launch_stream_r<T, 1, DERIV, SG, BALL>(a, s);
  if (a.run == 2) return launch_stream_r<T, 2, DERIV, SG, BALL>(a, s);
  if constexpr (sizeof(T) == 4)
    if (a.run == 4) return launch_stream_r<T, 4, DERIV, SG, BALL>(a, s);
  return hipErrorInvalidValue;
}

template <typename T, int DERIV>
hipError_t launch_stream_d(const StreamArgs<T> &a, bool ball, hipStream_t s) {
  bool sg = a.sg[0] != T(0) || a.sg[1] != T(0);
  if (ball) return sg ? launch_stream_v<T, DERIV, true, true>(a, s) : launch_stream_v<T, DERIV, false, true>(a, s);
  return sg ? launch_stream_v<T, DERIV, true, false>(a, s) : launch_stream_v<T, DERIV, false, false>(a, s);
}

template <typename T, int R, int DERIV, bool SG, bool BALL, bool SEG, bool RANGE, bool ROWS2 = false>
void launch_plane_form(const StreamArgs<T> &a, unsigned blocks, int threads, size_t lds, hipStream_t s) {
  // the compiled-in forms (not for the ball test dynamics); the 4D clamp
  // target, and the eps fold other than in TVD-RK2 stage 2 of one-row
  // blocks, take the runtime form
  int form = kFormRuntime;
  if (RANGE)
    form = kFormPlain;
  else if (!BALL && !a.eps) {
    if (a.mode == kPlain && !a.clamp)
      form = kFormPlain;
    else if (a.mode == kPlain && a.clamp && a.v0xy)
      form = kFormPlainXY;
    else if (a.mode == kAverage && a.clamp && a.v0xy)
      form = kFormAverageXY;
  } else if (!BALL && !ROWS2 && a.mode == kAverage && a.clamp && a.v0xy) {
    form = kFormAverageXYEps;  // a.eps set
  }
  if (form == kFormPlain)
    hipLaunchKernelGGL((stage_plane<T, R, DERIV, SG, BALL, SEG, RANGE, kFormPlain, ROWS2>), dim3(blocks),
                       dim3(threads), lds, s, a);
  else if constexpr (!RANGE && !BALL) {
    if (form == kFormPlainXY)
      hipLaunchKernelGGL((stage_plane<T, R, DERIV, SG, BALL, SEG, false, kFormPlainXY, ROWS2>), dim3(blocks),
                         dim3(threads), lds, s, a);
    else if (form == kFormAverageXY)
      hipLaunchKernelGGL((stage_plane<T, R, DERIV, SG, BALL, SEG, false, kFormAverageXY, ROWS2>), dim3(blocks),
                         dim3(threads), lds, s, a);
    else if (form == kFormAverageXYEps && !ROWS2)
      hipLaunchKernelGGL((stage_plane<T, R, DERIV, SG, BALL, SEG, false, kFormAverageXYEps, false>), dim3(blocks),
                         dim3(threads), lds, s, a);
    else
      hipLaunchKernelGGL((stage_plane<T, R, DERIV, SG, BALL, SEG, false, kFormRuntime, ROWS2>), dim3(blocks),
                         dim3(threads), lds, s, a);
  } else if constexpr (!RANGE) {
    hipLaunchKernelGGL((stage_plane<T, R, DERIV, SG, BALL, SEG, false, kFormRuntime>), dim3(blocks), dim3(threads),
                       lds, s, a);
  }
}

template <typename T, int R, int DERIV, bool SG, bool BALL, bool RANGE = false>
hipError_t launch_plane_r(const StreamArgs<T> &a, hipStream_t s) {
  const bool seg = a.n_seg > 1;
  const bool rows2 = a.rows == 2;
  const int rows = seg ? a.v_seg : a.n[2];
  const int runs = rows * a.runs_per_row;
  constexpr int SL = R == 3 ? 4 : R;  // LDS elements per run
  // ragged rows (runs of 2 or 4, whole planes): ceil(N_theta / R) runs, N_theta >= 2 R
  const bool ragged_ok = (R == 2 || R == 4) && !seg && a.n[3] >= 2 * R && a.runs_per_row == (a.n[3] + R - 1) / R;
  // two-row blocks: each row's runs in whole waves, an even number of rows,
  // chunk mode, the stage only
  const int threads = rows2 ? 2 * ((runs + 63) / 64 * 64) : (runs + 63) / 64 * 64;
  if (threads > (R == 3 ? kPlaneMaxThreads3 : kPlaneMaxThreads) || a.run != R || a.span < 0 || (a.span && seg) ||
      (a.runs_per_row * R != a.n[3] && !ragged_ok) || (R == 3 && seg) ||
      (a.rows != 0 && a.rows != 1 && !rows2) ||
      (rows2 && (RANGE || BALL || a.span || a.n[1] % 2 != 0)) ||
      a.blocks_per_chunk != a.n[1] / (rows2 ? 2 : 1) * (seg ? a.n_seg : 1) ||
      (seg && (a.v_seg < kPlaneMinSegRows || (int64_t)a.v_seg * a.n_seg < a.n[2] ||
               (int64_t)a.v_seg * (a.n_seg - 1) >= a.n[2])))
    return hipErrorInvalidValue;
  // two buffers of the plane (or of the segment and its halo rows) per row;
  // two-row blocks add two buffers of the published neighbours per row
  const size_t plane_lds = 2 * (size_t)(seg ? a.v_seg + 4 : a.n[2]) * a.runs_per_row * SL * sizeof(T);
  const size_t lds = rows2 ? 2 * plane_lds + 4 * (size_t)rows * a.runs_per_row * SL * sizeof(T) : plane_lds;
  if (lds > (size_t)kPlaneMaxLdsBytes) return hipErrorInvalidValue;
  const unsigned blocks = a.span ? (unsigned)a.span : (unsigned)(a.blocks_per_chunk * a.n_chunks);
  if constexpr (!RANGE && !BALL) {
    if (rows2) {
      if (seg && R != 3)
        launch_plane_form<T, R, DERIV, SG, BALL, R != 3, false, true>(a, blocks, threads, lds, s);
      else
        launch_plane_form<T, R, DERIV, SG, BALL, false, false, true>(a, blocks, threads, lds, s);
      return hipGetLastError();
    }
  }
  if constexpr (R == 3) {
    launch_plane_form<T, R, DERIV, SG, BALL, false, RANGE>(a, blocks, threads, lds, s);
  } else {
    if (seg)
      launch_plane_form<T, R, DERIV, SG, BALL, true, RANGE>(a, blocks, threads, lds, s);
    else
      launch_plane_form<T, R, DERIV, SG, BALL, false, RANGE>(a, blocks, threads, lds, s);
  }
  return hipGetLastError();
}



template <typename T, int DERIV, bool SG, bool BALL>
hipError_t launch_plane_v(const StreamArgs<T> &a, hipStream_t s) {
  if (a.run == 1) return launch_plane_r<T, 1, DERIV, SG, BALL>(a, s);
  if (a.run == 2) return launch_plane_r<T, 2, DERIV, SG, BALL>(a, s);
  if constexpr (sizeof(T) == 4) {
    if (a.run == 4) return launch_plane_r<T, 4, DERIV, SG, BALL>(a, s);
    if (a.run == 3) return launch_plane_r<T, 3, DERIV, SG, BALL>(a, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, int DERIV>
hipError_t launch_plane_d(const StreamArgs<T> &a, bool ball, hipStream_t s) {
  bool sg = a.sg[0] != T(0) || a.sg[1] != T(0);
  if (ball) return sg ? launch_plane_v<T, DERIV, true, true>(a, s) : launch_plane_v<T, DERIV, false, true>(a, s);
  return sg ? launch_plane_v<T, DERIV, true, false>(a, s) : launch_plane_v<T, DERIV, false, false>(a, s);
}

// ---------------------------------------------------------------------------
// Batched solves.  Every instance of a batch runs the streaming kernel's
// tiles; which arrays a tile reads and writes follows from its phase.
// ---------------------------------------------------------------------------

// The per-phase fields of instance `in` at step k, stage `stage`.
template <typename T>
__device__ inline void phase_args(StreamArgs<T> &a, const BatchInst<T> &in, int k, int stage) {
  const T *cur = k == 0 ? in.v0 : ((k & 1) ? in.vb : in.va);
  T *nxt = (k & 1) ? in.va : in.vb;
  a.dt = k == in.steps - 1 ? in.dt_last : in.dt;
  a.v0 = in.v0;
  if (!in.rk2) {
    a.vs = cur;
    a.vn = nullptr;
    a.out = nxt;
    a.mode = kPlain;
    a.clamp = in.clamp;
  } else if (stage == 0) {
    a.vs = cur;
    a.vn = nullptr;
    a.out = in.w1;
    a.mode = kPlain;
    a.clamp = 0;
  } else {
    a.vs = in.w1;
    a.vn = cur;
    a.out = nxt;
    a.mode = kAverage;
    a.clamp = in.clamp;
  }
}

// The run length differs between instances: dispatch inside the kernel (the
// choice is uniform over a block).
template <typename T, int DERIV, bool SG, bool BALL>
__device__ inline void tile_any_run(const StreamArgs<T> &a, int lb) {
  if (a.run == 1) {
    stream_tile<T, 1, DERIV, SG, BALL>(a, lb);
  } else if (a.run == 2) {
    stream_tile<T, 2, DERIV, SG, BALL>(a, lb);
  } else if constexpr (sizeof(T) == 4) {
    stream_tile<T, 4, DERIV, SG, BALL>(a, lb);
  }
}

// First j in [0, n) with end[j] > x (end ascending, end[n-1] > x).
__device__ inline int find_end(const int32_t *__restrict__ end, int n, int x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (end[mid] > x)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

template <typename T, int DERIV, bool SG, bool BALL>
__global__ __launch_bounds__(kStreamBlock) void stage_multi(const BatchInst<T> *__restrict__ inst,
                                                             const int32_t *__restrict__ tile_end, int ninst, int k,
                                                             int stage) {
  const int lb = (int)xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = find_end(tile_end, ninst, lb);
  StreamArgs<T> a = inst[j].a;
  phase_args(a, inst[j], k >= 0 ? k : inst[j].k + (-1 - k), stage);
  tile_any_run<T, DERIV, SG, BALL>(a, lb - (j > 0 ? tile_end[j - 1] : 0));
}

// The batched plane kernel: instance j's blocks run the plane kernel on its
// grid, at its own run length and with its own plane split, in the stage's
// runtime form.  A launch's blocks have as many work-items as its largest
// instance needs; the waves an instance leaves empty end at once, before
// any barrier (a workgroup barrier waits only for the waves that have not
// ended), so they hold no registers while the block sweeps its planes.
template <typename T, int DERIV, bool SG, bool BALL>
__global__ __launch_bounds__(kPlaneMaxThreads) void stage_plane_multi(const BatchInst<T> *__restrict__ inst,
                                                                      const int32_t *__restrict__ tile_end,
                                                                      int ninst, int k, int stage) {
  const int lb = (int)xcd_logical_block(blockIdx.x, gridDim.x);
  const int j = find_end(tile_end, ninst, lb);
  StreamArgs<T> a = inst[j].a;
  phase_args(a, inst[j], k >= 0 ? k : inst[j].k + (-1 - k), stage);
  const bool seg = a.n_seg > 1;
  // the block's runs: those of a whole plane, or of a full v segment (the
  // segment kernel's halo copy needs the work-items of 4 rows)
  const int runs = __builtin_amdgcn_readfirstlane((seg ? a.v_seg : a.n[2]) * a.runs_per_row);
  if (__builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6) * 64 >= runs) return;  // wave-uniform
  const int local = lb - (j > 0 ? tile_end[j - 1] : 0);
  const int nblk = inst[j].tiles;
  if (seg) {
    if (a.run == 2) plane_block<T, 2, DERIV, SG, BALL, true, false, kFormRuntime>(a, local, nblk);
  } else if (a.run == 2) {
    plane_block<T, 2, DERIV, SG, BALL, false, false, kFormRuntime>(a, local, nblk);
  } else if constexpr (sizeof(T) == 4) {
    if (a.run == 3)
      plane_block<T, 3, DERIV, SG, BALL, false, false, kFormRuntime>(a, local, nblk);
    else if (a.run == 4)
      plane_block<T, 4, DERIV, SG, BALL, false, false, kFormRuntime>(a, local, nblk);
  }
}

// The persistent batch kernel.  Each block takes work items in order from a
// global counter; an item is one tile of one instance in one phase.  Before
// a tile runs, every tile of the instance's previous phase must be complete
// (the tile reads x-, y-, v- and theta-neighbours that other tiles wrote),
// which the instance's completion counter shows.  Items are ordered by
// phase, so an item only waits for items taken before it, by blocks that are
// running: the queue always drains.  A wait gives up after spin_limit polls
// and raises the error flag, after which every block leaves, so the kernel
// ends in every case.
template <typename T, int DERIV, bool SG, bool BALL>
__global__ __launch_bounds__(kStreamBlock) void stage_persistent(PersistArgs<T> p) {
  __shared__ int32_t s_item, s_abort;
  BatchQueue *q = p.queue;
  const int32_t total = p.start[p.nphase];
  int ph = 0;  // phase of the last item (items of a block only increase)
  for (;;) {
    if (threadIdx.x == 0) s_item = __hip_atomic_fetch_add(&q->next, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int32_t item = s_item;
    if (item >= total) break;
    while (item >= p.start[ph + 1]) ++ph;
    const int32_t local = item - p.start[ph];
    const int j = find_end(p.tile_end, p.active[ph], local);
    const int tile = local - (j > 0 ? p.tile_end[j - 1] : 0);
    if (threadIdx.x == 0) {
      const int32_t need = ph * p.inst[j].tiles;
      int ok = 1;
      int64_t spins = 0;
      while (__hip_atomic_load(&q->done[j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
        if (__hip_atomic_load(&q->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++spins > p.spin_limit) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      if (!ok) __hip_atomic_store(&q->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_abort = !ok;
      // the acquire above invalidated this CU's L1 and the stale L2 lines
      // for the whole block; the barrier orders the other waves' loads after it
    }
    __syncthreads();
    if (s_abort) break;
    StreamArgs<T> a = p.inst[j].a;
    phase_args(a, p.inst[j], ph / p.phases_per_step, ph % p.phases_per_step);
    tile_any_run<T, DERIV, SG, BALL>(a, tile);
    // every wave's stores complete, then one agent-scope release (L2
    // write-back) publishes the block's tile with the counter
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(&q->done[j], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void batch_reset_kernel(BatchQueue *q, int m) {
  for (int i = threadIdx.x; i < m; i += blockDim.x) q->done[i] = 0;
  if (threadIdx.x == 0) {
    q->next = 0;
    q->error = 0;
  }
}

// ---------------------------------------------------------------------------
// Algorithm 1's derivative range: the smallest and largest derivative per
// axis over the grid -- of the central derivative (p- + p+) / 2 of eq (5),
// or (range_onesided) of both one-sided derivatives.  Doubles are compared through an
// order-preserving 64-bit key (sign bit flipped for non-negative values,
// all bits flipped for negative ones), so unsigned atomics give min and max.
// ---------------------------------------------------------------------------


constexpr int kRangeXSeg = 16;  // x planes per thread in the derivative-range pass

template <typename T, int DERIV>
__global__ __launch_bounds__(256) void deriv_range_kernel(StageArgs<T> a, unsigned long long *keys) {
  __shared__ unsigned long long part[8][4];
  T lo[4], hi[4];  // min and max are exact in T; widened for the keys
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    lo[d] = T(INFINITY);
    hi[d] = T(-INFINITY);
  }
  // A thread takes an x segment of one (y, v, theta) column: the column's
  // index is split once and the node moves by one x plane per iteration.
  // Where every axis's window lies on the grid (or wraps on a periodic
  // axis) the window values are loads at offsets fixed for the thread, and
  // the loop is unrolled so that several nodes' loads are in flight at once;
  // windows that need extrapolated ghosts go through axis_value.  Node
  // indices fit 32 bits (grids have fewer than 2^31 nodes).
  constexpr int RW = DERIV == kUpwind1 ? 1 : 2;
  const int cols = (int)a.st[0];  // n[1] n[2] n[3]
  const int nx = a.n[0];
  const int nseg = (nx + kRangeXSeg - 1) / kRangeXSeg;
  const bool onesided = a.range_onesided != 0;
  auto reduce = [&](int d, T pm, T pp) {
    const T cen = T(0.5) * (pm + pp);
    const T mn = onesided ? (pm < pp ? pm : pp) : cen, mx = onesided ? (pm < pp ? pp : pm) : cen;
    lo[d] = mn < lo[d] ? mn : lo[d];
    hi[d] = mx > hi[d] ? mx : hi[d];
  };
  for (int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; item < (int64_t)cols * nseg;
       item += (int64_t)gridDim.x * blockDim.x) {
    const int seg = (int)(item / cols), col = (int)(item - (int64_t)seg * cols);
    int idx[4];
    idx[3] = col % a.n[3];
    idx[2] = (col / a.n[3]) % a.n[2];
    idx[1] = col / (a.n[3] * a.n[2]);
    int off[4][5];
    bool direct = true;
#pragma unroll
    for (int d = 1; d < 4; ++d) {
      const bool per = (a.periodic_mask >> d) & 1u;
      direct = direct && (per || (idx[d] >= RW && idx[d] + RW < a.n[d]));
#pragma unroll
      for (int o = -2; o <= 2; ++o) {
        int t = idx[d] + o;
        t = t < 0 ? t + a.n[d] : (t >= a.n[d] ? t - a.n[d] : t);
        off[d][o + 2] = (t - idx[d]) * (int)a.st[d];
      }
    }
#pragma unroll
    for (int o = -2; o <= 2; ++o) off[0][o + 2] = o * cols;
    const int xa = seg * kRangeXSeg, xb = min(nx, xa + kRangeXSeg);
    // the x range whose windows are all plain loads
    const int fa = direct ? max(xa, RW) : xb, fb = direct ? min(xb, nx - RW) : xb;
    for (int x = xa; x < xb; ++x) {
      if (x == fa && fa < fb) {
#pragma unroll 4
        for (int xf = fa; xf < fb; ++xf) {
          const int p = xf * cols + col;
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            T w[5], pm, pp;
#pragma unroll
            for (int o = -2; o <= 2; ++o) w[o + 2] = (o < -RW || o > RW) ? T(0) : a.vs[p + off[d][o + 2]];
            one_sided<T, DERIV>(w, a.inv_h[d], pm, pp);
            reduce(d, pm, pp);
          }
        }
        x = fb - 1;
        continue;
      }
      idx[0] = x;
      const int p = x * cols + col;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        T w[5], pm, pp;
        const bool per = (a.periodic_mask >> d) & 1u;
#pragma unroll
        for (int o = -2; o <= 2; ++o)
          w[o + 2] = (o < -RW || o > RW) ? T(0) : axis_value(a.vs, p, idx[d], o, a.n[d], a.st[d], per);
        one_sided<T, DERIV>(w, a.inv_h[d], pm, pp);
        reduce(d, pm, pp);
      }
    }
  }
  // block reduction in key space: min of the lows, max of the highs
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    unsigned long long kl = order_key((double)lo[d]), kh = order_key((double)hi[d]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      unsigned long long ol = __shfl_xor(kl, o, 64), oh = __shfl_xor(kh, o, 64);
      kl = ol < kl ? ol : kl;
      kh = oh > kh ? oh : kh;
    }
    if (lane == 0) {
      part[d][wave] = kl;
      part[4 + d][wave] = kh;
    }
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int d = threadIdx.x;
    unsigned long long kl = part[d][0], kh = part[4 + d][0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      kl = part[d][w] < kl ? part[d][w] : kl;
      kh = part[4 + d][w] > kh ? part[4 + d][w] : kh;
    }
    unsigned long long *set = keys + 8 * (blockIdx.x % kRangeSlots);
    atomicMin(&set[d], kl);
    atomicMax(&set[4 + d], kh);
  }
}

__global__ void range_reset_kernel(unsigned long long *keys) {
  for (int i = threadIdx.x; i < 8 * kRangeSlots; i += blockDim.x) keys[i] = (i & 7) < 4 ? ~0ull : 0ull;
}

// ---------------------------------------------------------------------------
// Convergence mode: the largest change of a step, and the stop test.
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void delta_max_kernel(const T *__restrict__ a, const T *__restrict__ b, int64_t n,
                                                        int64_t nvec, unsigned long long *acc, const int32_t *skip) {
  if (skip && *skip) return;
  __shared__ double part[4];
  double m = 0.0;
  // |a - b| in FP64 (exact for FP32 inputs); NaN counts as infinitely large
  auto take = [&](T x, T y) {
    double d = fabs((double)x - (double)y);
    if (d != d) d = INFINITY;
    m = d > m ? d : m;
  };
  // nvec 16-byte vectors (both arrays 16-byte aligned, else nvec = 0), then
  // the remaining elements one by one
  constexpr int VW = 16 / (int)sizeof(T);
  typedef typename VecT<T, VW>::type V;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride) {
    const V x = reinterpret_cast<const V *>(a)[i], y = reinterpret_cast<const V *>(b)[i];
#pragma unroll
    for (int j = 0; j < VW; ++j) take(x[j], y[j]);
  }
  for (int64_t i = nvec * VW + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) take(a[i], b[i]);
  m = wave_max_d(m);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = part[w] > m ? part[w] : m;
    atomicMax(acc, (unsigned long long)__double_as_longlong(m));  // non-negative: bit order = value order
  }
}

__global__ void converge_check_kernel(unsigned long long *acc, double threshold, int32_t *state, double *eps_log,
                                      int slot, int64_t k) {
  if (state[0]) return;
  double eps = __longlong_as_double((long long)*acc);
  eps_log[slot] = eps;
  *acc = 0ull;
  if (eps < threshold) {
    state[0] = 1;
    state[1] = (int32_t)(k + 1);
  }
}

__global__ void converge_reset_kernel(unsigned long long *acc, int32_t *state) {
  *acc = 0ull;
  state[0] = 0;
  state[1] = 0;
}

// ---------------------------------------------------------------------------
// Optimal control at arbitrary states (eq (9)): grad V and V at the state by
// multilinear interpolation over the 16 corners of its cell, of the nodal
// central-difference gradient (one-sided at the ends of an open axis, wrapped
// on a periodic one) and of V; then the bang-bang control.  FP64 whatever the
// grid's precision; no fused multiply-add, in a fixed order (corners with the
// theta bit fastest, weights multiplied x, y, v, theta), so that the result
// is reproducible from the same V.
// ---------------------------------------------------------------------------

template <typename T>
__device__ inline double node_value(const ControlArgs<T> &a, const int (&idx)[4]) {
  int64_t off = (((int64_t)idx[0] * a.n[1] + idx[1]) * a.n[2] + idx[2]) * a.n[3] + idx[3];
  return (double)a.v[off];
}

template <typename T>
__device__ inline double node_gradient(const ControlArgs<T> &a, const int (&idx)[4], int d) {
#pragma clang fp contract(off)
  const int n = a.n[d], i = idx[d];
  int lo_i[4] = {idx[0], idx[1], idx[2], idx[3]}, hi_i[4] = {idx[0], idx[1], idx[2], idx[3]};
  double den;
  if ((a.periodic_mask >> d) & 1u) {
    lo_i[d] = i == 0 ? n - 1 : i - 1;
    hi_i[d] = i == n - 1 ? 0 : i + 1;
    den = 2.0 * a.h[d];
  } else if (i == 0) {
    hi_i[d] = 1;
    den = a.h[d];
  } else if (i == n - 1) {
    lo_i[d] = n - 2;
    den = a.h[d];
  } else {
    lo_i[d] = i - 1;
    hi_i[d] = i + 1;
    den = 2.0 * a.h[d];
  }
  return (node_value(a, hi_i) - node_value(a, lo_i)) / den;
}

template <typename T>
__global__ __launch_bounds__(64) void control_kernel(ControlArgs<T> a) {
#pragma clang fp contract(off)
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= a.m) return;
  const double *z = a.states + 4 * q;
  int i0[4], i1[4];
  double w[4];
  for (int d = 0; d < 4; ++d) {
    const int n = a.n[d];
    if ((a.periodic_mask >> d) & 1u) {
      double t = (z[d] - a.lo[d]) / a.h[d];
      t = fmod(t, (double)n);
      if (t < 0.0) t += (double)n;
      int c = (int)floor(t);
      if (c >= n) c = n - 1;
      i0[d] = c;
      i1[d] = c + 1 == n ? 0 : c + 1;
      w[d] = t - (double)c;
    } else {
      double s = z[d] < a.lo[d] ? a.lo[d] : (z[d] > a.hi[d] ? a.hi[d] : z[d]);
      double t = (s - a.lo[d]) / a.h[d];
      int c = (int)floor(t);
      if (c > n - 2) c = n - 2;
      if (c < 0) c = 0;
      i0[d] = c;
      i1[d] = c + 1;
      w[d] = t - (double)c;
    }
  }
  double val = 0.0, p[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c = 0; c < 16; ++c) {
    int idx[4];
    double wt = 1.0;
    for (int d = 0; d < 4; ++d) {
      const int bitd = (c >> (3 - d)) & 1;
      idx[d] = bitd ? i1[d] : i0[d];
      wt = wt * (bitd ? w[d] : 1.0 - w[d]);
    }
    val = val + wt * node_value(a, idx);
    for (int d = 0; d < 4; ++d) p[d] = p[d] + wt * node_gradient(a, idx, d);
  }
  a.controls[2 * q] = p[2] >= 0.0 ? a.a_max : -a.a_max;
  // the car turns at +-w_max by the sign of p_theta; the steering car steers
  // +-steer_max by the sign of p_theta v
  const double s3 = a.steer ? p[3] * z[2] : p[3];
  a.controls[2 * q + 1] = s3 >= 0.0 ? a.turn_max : -a.turn_max;
  if (a.values) a.values[q] = val;
  if (a.grads)
    for (int d = 0; d < 4; ++d) a.grads[4 * q + d] = p[d];
}

}  // namespace

template <typename T>
hipError_t launch_plane(const StreamArgs<T> &a, int deriv, bool ball, hipStream_t s) {
  if (deriv == kUpwind1) return launch_plane_d<T, kUpwind1>(a, ball, s);
  return launch_plane_d<T, kEno2>(a, ball, s);
}

template <typename T>
hipError_t launch_stream(const StreamArgs<T> &a, int deriv, bool ball, hipStream_t s) {
  if (deriv == kUpwind1) return launch_stream_d<T, kUpwind1>(a, ball, s);
  return launch_stream_d<T, kEno2>(a, ball, s);
}

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

template <typename T, int DERIV, bool SG, bool BALL>
static hipError_t launch_multi_v(const BatchInst<T> *inst, const int32_t *tile_end, int ninst, int blocks, int k,
                                 int stage, hipStream_t s) {
  hipLaunchKernelGGL((stage_multi<T, DERIV, SG, BALL>), dim3(blocks), dim3(kStreamBlock), 0, s, inst, tile_end, ninst,
                     k, stage);
  return hipGetLastError();
}

template <typename T>
bool plane_multi_fits(const StreamArgs<T> &a, int *threads, size_t *lds) {
  const int R = a.run;
  const bool seg = a.n_seg > 1;
  const bool run_ok = R == 2 || (sizeof(T) == 4 && (R == 3 || R == 4) && !seg);
  const bool ragged_ok = (R == 2 || R == 4) && !seg && a.n[3] >= 2 * R && a.runs_per_row == (a.n[3] + R - 1) / R;
  if (!run_ok || a.runs_per_row < 1 || (a.runs_per_row * R != a.n[3] && !ragged_ok) || a.span != 0 ||
      a.n_chunks < 1 ||
      a.chunk_len < 1 || (int64_t)a.chunk_len * a.n_chunks < a.n[0] ||
      (int64_t)a.chunk_len * (a.n_chunks - 1) >= a.n[0] || a.blocks_per_chunk != a.n[1] * (seg ? a.n_seg : 1))
    return false;
  if (seg && (a.v_seg < kPlaneMinSegRows || (int64_t)a.v_seg * a.n_seg < a.n[2] ||
              (int64_t)a.v_seg * (a.n_seg - 1) >= a.n[2]))
    return false;
  const int64_t runs = (int64_t)(seg ? a.v_seg : a.n[2]) * a.runs_per_row;
  const int64_t bytes = 2 * (int64_t)(seg ? a.v_seg + 4 : a.n[2]) * a.runs_per_row * (R == 3 ? 4 : R) * sizeof(T);
  if (runs > kPlaneMaxThreads || bytes > kPlaneMaxLdsBytes) return false;
  *threads = (int)((runs + 63) / 64 * 64);
  *lds = (size_t)bytes;
  return true;
}

template <typename T, int DERIV, bool SG, bool BALL>
static hipError_t launch_plane_multi_v(const BatchInst<T> *inst, const int32_t *tile_end, int ninst, int blocks,
                                       int threads, size_t lds, int k, int stage, hipStream_t s) {
  hipLaunchKernelGGL((stage_plane_multi<T, DERIV, SG, BALL>), dim3(blocks), dim3(threads), lds, s, inst, tile_end,
                     ninst, k, stage);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_plane_multi(const BatchInst<T> *inst, const int32_t *tile_end, int ninst, int blocks, int threads,
                              size_t lds, int k, int stage, int deriv, bool sg, bool ball, hipStream_t s) {
  if (blocks < 1 || ninst < 1 || threads < 64 || threads > kPlaneMaxThreads || threads % 64 != 0 ||
      lds > (size_t)kPlaneMaxLdsBytes)
    return hipErrorInvalidValue;
#define HJ_PMULTI(D, G, B) \
  return launch_plane_multi_v<T, D, G, B>(inst, tile_end, ninst, blocks, threads, lds, k, stage, s)
  if (deriv == kUpwind1) {
    if (ball) {
      if (sg) HJ_PMULTI(kUpwind1, true, true);
      HJ_PMULTI(kUpwind1, false, true);
    }
    if (sg) HJ_PMULTI(kUpwind1, true, false);
    HJ_PMULTI(kUpwind1, false, false);
  }
  if (ball) {
    if (sg) HJ_PMULTI(kEno2, true, true);
    HJ_PMULTI(kEno2, false, true);
  }
  if (sg) HJ_PMULTI(kEno2, true, false);
  HJ_PMULTI(kEno2, false, false);
#undef HJ_PMULTI
}

template <typename T>
hipError_t launch_multi(const BatchInst<T> *inst, const int32_t *tile_end, int ninst, int blocks, int k, int stage,
                        int deriv, bool sg, bool ball, hipStream_t s) {
#define HJ_MULTI(D, G, B) return launch_multi_v<T, D, G, B>(inst, tile_end, ninst, blocks, k, stage, s)
  if (deriv == kUpwind1) {
    if (ball) {
      if (sg) HJ_MULTI(kUpwind1, true, true);
      HJ_MULTI(kUpwind1, false, true);
    }
    if (sg) HJ_MULTI(kUpwind1, true, false);
    HJ_MULTI(kUpwind1, false, false);
  }
  if (ball) {
    if (sg) HJ_MULTI(kEno2, true, true);
    HJ_MULTI(kEno2, false, true);
  }
  if (sg) HJ_MULTI(kEno2, true, false);
  HJ_MULTI(kEno2, false, false);
#undef HJ_MULTI
}

template <typename T, int DERIV, bool SG, bool BALL>
static hipError_t launch_persistent_v(const PersistArgs<T> &p, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((stage_persistent<T, DERIV, SG, BALL>), dim3(blocks), dim3(kStreamBlock), 0, s, p);
  return hipGetLastError();
}

template <typename T, int DERIV, bool SG, bool BALL>
static int persistent_occupancy() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, stage_persistent<T, DERIV, SG, BALL>, kStreamBlock, 0) !=
      hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

template <typename T>
hipError_t launch_persistent(const PersistArgs<T> &p, int blocks, int deriv, bool sg, bool ball, hipStream_t s) {
#define HJ_PERS(D, G, B) return launch_persistent_v<T, D, G, B>(p, blocks, s)
  if (deriv == kUpwind1) {
    if (ball) {
      if (sg) HJ_PERS(kUpwind1, true, true);
      HJ_PERS(kUpwind1, false, true);
    }
    if (sg) HJ_PERS(kUpwind1, true, false);
    HJ_PERS(kUpwind1, false, false);
  }
  if (ball) {
    if (sg) HJ_PERS(kEno2, true, true);
    HJ_PERS(kEno2, false, true);
  }
  if (sg) HJ_PERS(kEno2, true, false);
  HJ_PERS(kEno2, false, false);
#undef HJ_PERS
}

template <typename T>
int persistent_blocks_per_cu(int deriv, bool sg, bool ball) {
#define HJ_OCC(D, G, B) return persistent_occupancy<T, D, G, B>()
  if (deriv == kUpwind1) {
    if (ball) {
      if (sg) HJ_OCC(kUpwind1, true, true);
      HJ_OCC(kUpwind1, false, true);
    }
    if (sg) HJ_OCC(kUpwind1, true, false);
    HJ_OCC(kUpwind1, false, false);
  }
  if (ball) {
    if (sg) HJ_OCC(kEno2, true, true);
    HJ_OCC(kEno2, false, true);
  }
  if (sg) HJ_OCC(kEno2, true, false);
  HJ_OCC(kEno2, false, false);
#undef HJ_OCC
}

hipError_t launch_batch_reset(BatchQueue *queue, int m, hipStream_t s) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(256), 0, s, queue, m);
  return hipGetLastError();
}

template hipError_t launch_multi<float>(const BatchInst<float> *, const int32_t *, int, int, int, int, int, bool, bool,
                                        hipStream_t);
template hipError_t launch_multi<double>(const BatchInst<double> *, const int32_t *, int, int, int, int, int, bool,
                                         bool, hipStream_t);
template hipError_t launch_plane_multi<float>(const BatchInst<float> *, const int32_t *, int, int, int, size_t, int,
                                              int, int, bool, bool, hipStream_t);
template hipError_t launch_plane_multi<double>(const BatchInst<double> *, const int32_t *, int, int, int, size_t, int,
                                               int, int, bool, bool, hipStream_t);
template bool plane_multi_fits<float>(const StreamArgs<float> &, int *, size_t *);
template bool plane_multi_fits<double>(const StreamArgs<double> &, int *, size_t *);
template hipError_t launch_persistent<float>(const PersistArgs<float> &, int, int, bool, bool, hipStream_t);
template hipError_t launch_persistent<double>(const PersistArgs<double> &, int, int, bool, bool, hipStream_t);
template int persistent_blocks_per_cu<float>(int, bool, bool);
template int persistent_blocks_per_cu<double>(int, bool, bool);
template <typename T>
hipError_t launch_delta_max(const T *a, const T *b, int64_t n, unsigned long long *acc, const int32_t *skip,
                            hipStream_t s) {
  const int64_t vw = 16 / (int64_t)sizeof(T);
  const int64_t nvec = (((uintptr_t)a | (uintptr_t)b) & 15) == 0 ? n / vw : 0;
  int64_t blocks = ((nvec > 0 ? nvec : n) + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(delta_max_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, a, b, n, nvec, acc, skip);
  return hipGetLastError();
}

hipError_t launch_converge_check(unsigned long long *acc, double threshold, int32_t *state, double *eps_log, int slot,
                                 int64_t k, hipStream_t s) {
  hipLaunchKernelGGL(converge_check_kernel, dim3(1), dim3(1), 0, s, acc, threshold, state, eps_log, slot, k);
  return hipGetLastError();
}

hipError_t launch_converge_reset(unsigned long long *acc, int32_t *state, hipStream_t s) {
  hipLaunchKernelGGL(converge_reset_kernel, dim3(1), dim3(1), 0, s, acc, state);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_control(const ControlArgs<T> &a, hipStream_t s) {
  if (a.m <= 0) return hipSuccess;
  hipLaunchKernelGGL(control_kernel<T>, dim3((unsigned)((a.m + 63) / 64)), dim3(64), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_delta_max<float>(const float *, const float *, int64_t, unsigned long long *,
                                            const int32_t *, hipStream_t);
template hipError_t launch_delta_max<double>(const double *, const double *, int64_t, unsigned long long *,
                                             const int32_t *, hipStream_t);
template hipError_t launch_control<float>(const ControlArgs<float> &, hipStream_t);
template hipError_t launch_control<double>(const ControlArgs<double> &, hipStream_t);
template <typename T>
hipError_t launch_deriv_range(const StageArgs<T> &a, int deriv, unsigned long long *keys, hipStream_t s) {
  hipLaunchKernelGGL(range_reset_kernel, dim3(1), dim3(256), 0, s, keys);
  const int64_t items = a.st[0] * ((a.n[0] + kRangeXSeg - 1) / kRangeXSeg);  // (column, x segment) pairs
  int64_t blocks = (items + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (deriv == kUpwind1)
    hipLaunchKernelGGL((deriv_range_kernel<T, kUpwind1>), dim3((unsigned)blocks), dim3(256), 0, s, a, keys);
  else
    hipLaunchKernelGGL((deriv_range_kernel<T, kEno2>), dim3((unsigned)blocks), dim3(256), 0, s, a, keys);
  return hipGetLastError();
}

template hipError_t launch_deriv_range<float>(const StageArgs<float> &, int, unsigned long long *, hipStream_t);
template hipError_t launch_deriv_range<double>(const StageArgs<double> &, int, unsigned long long *, hipStream_t);
template hipError_t launch_stream<float>(const StreamArgs<float> &, int, bool, hipStream_t);
template hipError_t launch_plane<float>(const StreamArgs<float> &, int, bool, hipStream_t);
template hipError_t launch_plane<double>(const StreamArgs<double> &, int, bool, hipStream_t);
template hipError_t launch_stream<double>(const StreamArgs<double> &, int, bool, hipStream_t);
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

// The derivative-range pass on the plane kernel's traversal (the one-sided
// differences it computes for a stage, reduced instead of combined): a.vs =
// V, a.range = kRangeSlots key sets, reset here; nothing else is written.
template <typename T>
hipError_t launch_plane_range(StreamArgs<T> a, int deriv, hipStream_t s) {
  if (!a.range) return hipErrorInvalidValue;
  a.mode = kPlain;
  a.clamp = 0;
  a.eps = nullptr;
  a.out = nullptr;
  hipLaunchKernelGGL(range_reset_kernel, dim3(1), dim3(256), 0, s, a.range);
  auto by_run = [&](auto deriv_c) -> hipError_t {
    constexpr int D = decltype(deriv_c)::value;
    if (a.run == 1) return launch_plane_r<T, 1, D, false, false, true>(a, s);
    if (a.run == 2) return launch_plane_r<T, 2, D, false, false, true>(a, s);
    if constexpr (sizeof(T) == 4) {
      if (a.run == 4) return launch_plane_r<T, 4, D, false, false, true>(a, s);
      if (a.run == 3) return launch_plane_r<T, 3, D, false, false, true>(a, s);
    }
    return hipErrorInvalidValue;
  };
  if (deriv == kUpwind1) return by_run(std::integral_constant<int, kUpwind1>());
  return by_run(std::integral_constant<int, kEno2>());
}

template hipError_t launch_plane_range<float>(StreamArgs<float>, int, hipStream_t);
template hipError_t launch_plane_range<double>(StreamArgs<double>, int, hipStream_t);

}  // namespace hj
