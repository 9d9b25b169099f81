/*
 * hj_oracle.c -- plain, slow, FP64 CPU reference for one explicit time step
 * of the grid Hamilton-Jacobi reachability PDE (Backward Reachable Tube of a
 * 4D car), written from the paper "Real-Time Formal Verification of
 * Autonomous Systems With An FPGA" (arXiv 2012.04011).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker that the HIP library is
 * compared against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or constant
 * with the HIP library: every quantity below is recomputed here from its
 * definition.
 *
 * What is computed (paper section "Basic Numerical Solution", Algorithm 2,
 * with the readings listed at each function):
 *   - nodes of a 4D grid (axes x, y, v, theta; theta periodic);
 *   - the cone/cylinder target V0 of eq (7), generalised to a union (min);
 *   - the dissipation coefficients alpha_d(z) and the CFL step
 *     dt = cfl / sum_d(alpha_d^max / dx_d)  (Algorithm 1, step-bound lines);
 *   - one-sided derivatives D-, D+ of eq (5) (first order) and the textbook
 *     second-order ENO variant (Osher & Shu 1991; Osher & Fedkiw 2003, s3.3);
 *   - the Hamiltonian H = grad(V) . f(z, u*, d*) with the control maximising
 *     and the disturbance minimising (eq 4), evaluated at the central
 *     derivative, plus Lax-Friedrichs dissipation with a '+' sign (the paper
 *     prints '-', which is anti-dissipative for this time direction);
 *   - forward Euler (Algorithm 2) or the two-stage TVD Runge-Kutta scheme
 *     (Shu & Osher 1988), followed by the clamp V = min(V0, V) (Algorithm 2,
 *     last line of the loop body; eq 4);
 *   - a fixed-horizon schedule: n = ceil(T / dt) steps, the last one shortened
 *     to T - (n - 1) dt.
 *
 * Layout: C order [x][y][v][theta], theta fastest (the paper's 4D array).
 * All arithmetic is IEEE binary64; build with -ffp-contract=off so that no
 * multiply-add is fused behind the reader's back.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { HJO_CAR4D = 0, HJO_DRIFT_INPUT = 1, HJO_CAR4D_STEER = 2 };
enum { HJO_UPWIND1 = 0, HJO_ENO2 = 1 };
enum { HJO_EULER = 0, HJO_TVD_RK2 = 1 };
enum { HJO_BOX = 0, HJO_BALL = 1 };
enum { HJO_INPUT_MAXIMIZES = 0, HJO_INPUT_MINIMIZES = 1 };

typedef struct {
  int32_t n[4];        /* nodes per axis: x, y, v, theta */
  double lo[4], hi[4]; /* axis ranges; for a periodic axis hi - lo is the period */
  uint32_t periodic_mask;
} hjo_grid;

/*
 * Dynamics.
 *   HJO_CAR4D:  x' = v cos(theta) + d_x, y' = v sin(theta) + d_y,
 *               v' = a, theta' = w; control (a, w) in a box, maximises;
 *               disturbance (d_x, d_y) in a box, minimises.
 *   HJO_DRIFT_INPUT (closed-form test cases):
 *               z' = drift + u, u nonzero only on the axes in in_axes_mask,
 *               bounded by in_speed in the box (per-axis) or Euclidean-ball
 *               norm; the input either maximises or minimises.
 *   HJO_CAR4D_STEER (the experiment's car, eq (6)): as HJO_CAR4D but
 *               theta' = v tan(delta) / L with the steering angle
 *               |delta| <= steer_max (< pi/2) and wheelbase L; control
 *               (a, delta) maximises.
 */
typedef struct {
  int32_t kind;
  double a_max, w_max, d_max[2];
  double drift[4], in_speed;
  uint32_t in_axes_mask;
  int32_t in_norm, in_role;
  double steer_max, wheelbase;
} hjo_dyn;

/* alpha_mode: HJO_ALPHA_STATE = alpha_d(z) bounds |f_d| over every input
 * (state-local, the default).  The other two are Algorithm 1's global
 * Lax-Friedrichs: alpha_d(z) = max |dH/dp_d (z, p)| over a box of gradients
 * found on the grid, axis by axis, recomputed every step together with dt.
 *   HJO_ALPHA_DERIV_RANGE: the box spans the smallest and largest central
 *     derivative D_d V = (D+ V + D- V) / 2 of eq (5) over the nodes, as
 *     Algorithm 1 prints it (the gradient at which H is evaluated).
 *   HJO_ALPHA_DERIV_RANGE_ONESIDED: the box spans every one-sided derivative
 *     (D- and D+ together), the textbook global Lax-Friedrichs bound: the
 *     numerical Hamiltonian is then monotone over every pair of one-sided
 *     values the grid holds, not only at each node's own average. */
enum { HJO_ALPHA_STATE = 0, HJO_ALPHA_DERIV_RANGE = 1, HJO_ALPHA_DERIV_RANGE_ONESIDED = 2 };

typedef struct {
  int32_t deriv, integrator, clamp, alpha_mode;
  double cfl;
} hjo_scheme;

/* ---------------------------------------------------------------- grid --- */

static int is_periodic(const hjo_grid *g, int d) { return (int)((g->periodic_mask >> d) & 1u); }

/* Node spacing: N nodes including both ends on an ordinary axis; N nodes over
 * one period on a periodic axis (theta_l = -pi + l * 2 pi / N). */
double hjo_spacing(const hjo_grid *g, int d) {
  if (is_periodic(g, d)) return (g->hi[d] - g->lo[d]) / g->n[d];
  return (g->hi[d] - g->lo[d]) / (g->n[d] - 1);
}

double hjo_node(const hjo_grid *g, int d, int i) { return g->lo[d] + i * hjo_spacing(g, d); }

int64_t hjo_num_points(const hjo_grid *g) {
  return (int64_t)g->n[0] * g->n[1] * g->n[2] * g->n[3];
}

static void strides_of(const hjo_grid *g, int64_t st[4]) {
  st[3] = 1;
  st[2] = g->n[3];
  st[1] = (int64_t)g->n[2] * g->n[3];
  st[0] = (int64_t)g->n[1] * g->n[2] * g->n[3];
}

static void unravel(const hjo_grid *g, int64_t p, int idx[4]) {
  for (int d = 3; d >= 0; --d) {
    idx[d] = (int)(p % g->n[d]);
    p /= g->n[d];
  }
}

/* ------------------------------------------------------------- target --- */

/* Eq (7) for a union of cylinders: distance in the (x, y) plane to each
 * obstacle centre minus its radius, minimum over obstacles; the same value
 * for every (v, theta). */
void hjo_target_cylinders(const hjo_grid *g, const double *cx, const double *cy, const double *r,
                          int32_t m, double *V0) {
  int64_t np = hjo_num_points(g);
  for (int64_t p = 0; p < np; ++p) {
    int idx[4];
    unravel(g, p, idx);
    double x = hjo_node(g, 0, idx[0]);
    double y = hjo_node(g, 1, idx[1]);
    double best = INFINITY;
    for (int o = 0; o < m; ++o) {
      double dist = sqrt((x - cx[o]) * (x - cx[o]) + (y - cy[o]) * (y - cy[o])) - r[o];
      if (dist < best) best = dist;
    }
    V0[p] = best;
  }
}

/* ------------------------------------------------------------ dynamics --- */

/* f(z, u, d) for the car; u = (a, w), dist = (d_x, d_y). */
static void car_f(double v, double theta, const double u[2], const double dist[2], double f[4]) {
  f[0] = v * cos(theta) + dist[0];
  f[1] = v * sin(theta) + dist[1];
  f[2] = u[0];
  f[3] = u[1];
}

/*
 * alpha_d(z) = max over all admissible controls and disturbances of
 * |f_d(z, u, d)| (state-local, independent of p).  The paper's Algorithm 2
 * uses |x'_d| at the optimal control; with a disturbance present that can be
 * smaller than the true bound and lose monotonicity, so the bound over the
 * whole input set is used.  For box sets the maximum of |affine| sits at a
 * vertex: |v cos(theta)| + d_x^max, |v sin(theta)| + d_y^max, a_max, w_max.
 * For the drift+input test dynamics: |drift_d| + speed on input axes (true
 * for both the box and the ball).
 */
static void alpha_at(const hjo_dyn *dy, const double z[4], double alpha[4]) {
  if (dy->kind == HJO_CAR4D || dy->kind == HJO_CAR4D_STEER) {
    alpha[0] = fabs(z[2] * cos(z[3])) + dy->d_max[0];
    alpha[1] = fabs(z[2] * sin(z[3])) + dy->d_max[1];
    alpha[2] = dy->a_max;
    /* tan is increasing on (-pi/2, pi/2): |v tan(delta) / L| peaks at the
     * largest steering angle */
    alpha[3] = dy->kind == HJO_CAR4D ? dy->w_max : fabs(z[2]) * tan(dy->steer_max) / dy->wheelbase;
  } else {
    for (int d = 0; d < 4; ++d) {
      alpha[d] = fabs(dy->drift[d]);
      if ((dy->in_axes_mask >> d) & 1u) alpha[d] += dy->in_speed;
    }
  }
}

/*
 * H(z, p) = p . f(z, u*, d*) with u* = argmax_u p.f (control) and
 * d* = argmin_d p.f (disturbance), eq (4) and eq (9).  Bang-bang on boxes;
 * ties (p_d = 0) take the '+' vertex for the control and the '-' vertex for
 * the disturbance -- the term they multiply is zero, so H does not depend on
 * the choice.
 */
static double hamiltonian(const hjo_dyn *dy, const double z[4], const double p[4]) {
  double f[4];
  if (dy->kind == HJO_CAR4D) {
    double u[2], dist[2];
    u[0] = p[2] >= 0.0 ? dy->a_max : -dy->a_max;
    u[1] = p[3] >= 0.0 ? dy->w_max : -dy->w_max;
    dist[0] = p[0] >= 0.0 ? -dy->d_max[0] : dy->d_max[0];
    dist[1] = p[1] >= 0.0 ? -dy->d_max[1] : dy->d_max[1];
    car_f(z[2], z[3], u, dist, f);
  } else if (dy->kind == HJO_CAR4D_STEER) {
    /* p_theta v tan(delta) / L is largest at delta = +-steer_max with the
     * sign of p_theta v (ties take +; the term is then zero) */
    double u[2], dist[2];
    u[0] = p[2] >= 0.0 ? dy->a_max : -dy->a_max;
    double delta = p[3] * z[2] >= 0.0 ? dy->steer_max : -dy->steer_max;
    u[1] = z[2] * tan(delta) / dy->wheelbase;
    dist[0] = p[0] >= 0.0 ? -dy->d_max[0] : dy->d_max[0];
    dist[1] = p[1] >= 0.0 ? -dy->d_max[1] : dy->d_max[1];
    car_f(z[2], z[3], u, dist, f);
  } else {
    double sgn = dy->in_role == HJO_INPUT_MAXIMIZES ? 1.0 : -1.0;
    double u[4] = {0.0, 0.0, 0.0, 0.0};
    if (dy->in_norm == HJO_BOX) {
      for (int d = 0; d < 4; ++d)
        if ((dy->in_axes_mask >> d) & 1u) u[d] = sgn * (p[d] >= 0.0 ? dy->in_speed : -dy->in_speed);
    } else {
      double norm2 = 0.0;
      for (int d = 0; d < 4; ++d)
        if ((dy->in_axes_mask >> d) & 1u) norm2 += p[d] * p[d];
      double norm = sqrt(norm2);
      if (norm > 0.0)
        for (int d = 0; d < 4; ++d)
          if ((dy->in_axes_mask >> d) & 1u) u[d] = sgn * dy->in_speed * p[d] / norm;
    }
    for (int d = 0; d < 4; ++d) f[d] = dy->drift[d] + u[d];
  }
  return p[0] * f[0] + p[1] * f[1] + p[2] * f[2] + p[3] * f[3];
}

/* Exported for tests: H and alpha at an arbitrary state and gradient. */
double hjo_hamiltonian(const hjo_dyn *dy, const double z[4], const double p[4]) {
  return hamiltonian(dy, z, p);
}
void hjo_alpha(const hjo_dyn *dy, const double z[4], double alpha[4]) { alpha_at(dy, z, alpha); }

/* ------------------------------------------------------------ CFL step --- */

/* alpha_d^max = max over every grid node of alpha_d(z) (Algorithm 1). */
void hjo_alpha_max(const hjo_grid *g, const hjo_dyn *dy, double amax[4]) {
  for (int d = 0; d < 4; ++d) amax[d] = 0.0;
  int64_t np = hjo_num_points(g);
  for (int64_t p = 0; p < np; ++p) {
    int idx[4];
    double z[4], a[4];
    unravel(g, p, idx);
    for (int d = 0; d < 4; ++d) z[d] = hjo_node(g, d, idx[d]);
    alpha_at(dy, z, a);
    for (int d = 0; d < 4; ++d)
      if (a[d] > amax[d]) amax[d] = a[d];
  }
}

/* dt = cfl / sum_d(alpha_d^max / dx_d); a zero sum (no motion at all) makes
 * one step of the whole horizon. */
double hjo_cfl_dt(const hjo_grid *g, const hjo_dyn *dy, double cfl, double horizon) {
  double amax[4];
  hjo_alpha_max(g, dy, amax);
  double s = 0.0;
  for (int d = 0; d < 4; ++d) s += amax[d] / hjo_spacing(g, d);
  if (s == 0.0) return horizon;
  return cfl / s;
}

/* Fixed horizon: n = ceil(T / dt); steps 1..n-1 take dt, the last takes
 * T - (n - 1) dt.  T = 0 means no step. */
void hjo_schedule(double dt, double horizon, int64_t *n_steps, double *dt_last) {
  if (horizon <= 0.0) {
    *n_steps = 0;
    *dt_last = 0.0;
    return;
  }
  int64_t n = (int64_t)ceil(horizon / dt);
  if (n < 1) n = 1;
  *n_steps = n;
  *dt_last = horizon - (double)(n - 1) * dt;
}

/* ------------------------------------------------------- derivatives --- */

/* Value at node idx shifted by `off` nodes along axis d.  Off the grid, a
 * periodic axis wraps; any other axis uses linear extrapolation from its two
 * end nodes ("extrapolated points" of eq (5)): the ghost k layers beyond an
 * end equals V_end + k (V_end - V_next). */
static double value_at(const hjo_grid *g, const double *V, const int64_t st[4], int64_t p,
                       const int idx[4], int d, int off) {
  int n = g->n[d];
  int i = idx[d] + off;
  int64_t base = p - (int64_t)idx[d] * st[d];
  if (i >= 0 && i < n) return V[base + (int64_t)i * st[d]];
  if (is_periodic(g, d)) {
    i = ((i % n) + n) % n;
    return V[base + (int64_t)i * st[d]];
  }
  if (i < 0) {
    double e = V[base], nx = V[base + st[d]];
    return e + (double)(-i) * (e - nx);
  }
  double e = V[base + (int64_t)(n - 1) * st[d]], nx = V[base + (int64_t)(n - 2) * st[d]];
  return e + (double)(i - (n - 1)) * (e - nx);
}

/*
 * One-sided derivatives along axis d at one node.
 *   UPWIND1 (eq 5):  p- = (V_i - V_{i-1}) / h,  p+ = (V_{i+1} - V_i) / h.
 *   ENO2 (textbook): with the undivided second difference in its
 *   divided-difference form, Q_j = (V_{j+1} - V_j) - (V_j - V_{j-1}),
 *     p- = (V_i - V_{i-1}) / h + c- / (2h),  c- = the smaller-magnitude of
 *          Q_{i-1}, Q_i (ties pick Q_{i-1});
 *     p+ = (V_{i+1} - V_i) / h - c+ / (2h),  c+ = the smaller-magnitude of
 *          Q_i, Q_{i+1} (ties pick Q_i).
 */
static void one_sided(const hjo_grid *g, int deriv, const double *V, const int64_t st[4], int64_t p,
                      const int idx[4], int d, double *pm, double *pp) {
  double h = hjo_spacing(g, d);
  if (deriv == HJO_UPWIND1) {
    double vm = value_at(g, V, st, p, idx, d, -1);
    double v0 = V[p];
    double vp = value_at(g, V, st, p, idx, d, +1);
    *pm = (v0 - vm) / h;
    *pp = (vp - v0) / h;
    return;
  }
  double w[5];
  for (int k = -2; k <= 2; ++k) w[k + 2] = value_at(g, V, st, p, idx, d, k);
  double d0 = w[1] - w[0], d1 = w[2] - w[1], d2 = w[3] - w[2], d3 = w[4] - w[3];
  double q_left = d1 - d0;  /* Q_{i-1} */
  double q_mid = d2 - d1;   /* Q_i     */
  double q_right = d3 - d2; /* Q_{i+1} */
  double c_minus = fabs(q_left) <= fabs(q_mid) ? q_left : q_mid;
  double c_plus = fabs(q_mid) <= fabs(q_right) ? q_mid : q_right;
  *pm = d1 / h + c_minus / (2.0 * h);
  *pp = d2 / h - c_plus / (2.0 * h);
}

/* Exported for tests: p- and p+ along axis d at every node. */
void hjo_derivs(const hjo_grid *g, const hjo_scheme *sc, const double *V, int32_t d, double *pm,
                double *pp) {
  int64_t st[4];
  strides_of(g, st);
  int64_t np = hjo_num_points(g);
  for (int64_t p = 0; p < np; ++p) {
    int idx[4];
    unravel(g, p, idx);
    one_sided(g, sc->deriv, V, st, p, idx, d, &pm[p], &pp[p]);
  }
}

/* ------------------------------------------------------------ L(V) --- */

/* L(V)(z) = H(z, (p+ + p-)/2) + sum_d alpha_d(z) (p+_d - p-_d) / 2. */
/* ---------------------------------- Algorithm 1: derivative-range alpha --- */

/* Algorithm 1's minDeriv / maxDeriv per axis over every node of V: of the
 * central derivative (D+ + D-) / 2 (HJO_ALPHA_DERIV_RANGE), or of the two
 * one-sided derivatives together (HJO_ALPHA_DERIV_RANGE_ONESIDED). */
void hjo_deriv_range(const hjo_grid *g, const hjo_scheme *sc, const double *V, double pmin[4], double pmax[4]) {
  int64_t st[4];
  strides_of(g, st);
  int64_t np = hjo_num_points(g);
  for (int d = 0; d < 4; ++d) {
    pmin[d] = INFINITY;
    pmax[d] = -INFINITY;
  }
  for (int64_t p = 0; p < np; ++p) {
    int idx[4];
    unravel(g, p, idx);
    for (int d = 0; d < 4; ++d) {
      double a, b;
      one_sided(g, sc->deriv, V, st, p, idx, d, &a, &b);
      double lo, hi;
      if (sc->alpha_mode == HJO_ALPHA_DERIV_RANGE_ONESIDED) {
        lo = a < b ? a : b;
        hi = a < b ? b : a;
      } else {
        lo = hi = (b + a) / 2.0; /* D_d V of eq (5) */
      }
      if (lo < pmin[d]) pmin[d] = lo;
      if (hi > pmax[d]) pmax[d] = hi;
    }
  }
}

/* Largest |b + u| over the values u that a box-bounded input takes when its
 * gradient component runs over [lo, hi]: the input is +bound where p >= 0
 * and -bound where p < 0 (dir = +1; dir = -1 flips both), so the range
 * decides which of the two vertices occur. */
static double box_input_alpha(double b, double bound, int dir, double lo, double hi) {
  double up = dir * bound, dn = -dir * bound;  /* input at p >= 0, at p < 0 */
  double a = 0.0;
  if (hi >= 0.0) a = fabs(b + up);
  if (lo < 0.0 && fabs(b + dn) > a) a = fabs(b + dn);
  return a;
}

/* Range of p_d / |p_S| over the box (S = the ball's axes, d in S): it grows
 * with p_d; for p_d > 0 it falls as the other components grow, for p_d < 0
 * it rises.  A zero gradient counts as 0 (the input is then 0). */
static void ball_ratio_range(const double pmin[4], const double pmax[4], uint32_t mask, int d, double *gmin,
                             double *gmax) {
  double rmin2 = 0.0, rmax2 = 0.0;
  for (int e = 0; e < 4; ++e) {
    if (e == d || !((mask >> e) & 1u)) continue;
    double a = pmin[e] * pmin[e], b = pmax[e] * pmax[e];
    rmax2 += a > b ? a : b;
    if (!(pmin[e] <= 0.0 && pmax[e] >= 0.0)) rmin2 += a < b ? a : b;
  }
  double M = pmax[d], m = pmin[d];
  *gmax = M > 0.0 ? M / sqrt(M * M + rmin2) : (M < 0.0 ? M / sqrt(M * M + rmax2) : 0.0);
  *gmin = m < 0.0 ? m / sqrt(m * m + rmin2) : (m > 0.0 ? m / sqrt(m * m + rmax2) : 0.0);
}

/* alpha_d(z) = max over the gradient box of |dH/dp_d (z, p)| (Algorithm 1):
 * dH/dp_d = f_d(z, u*(p), d*(p)) for the input-affine dynamics here. */
void hjo_alpha_box(const hjo_dyn *dy, const double z[4], const double pmin[4], const double pmax[4],
                   double alpha[4]) {
  if (dy->kind == HJO_CAR4D || dy->kind == HJO_CAR4D_STEER) {
    /* the disturbance minimises: -d_max where p >= 0 */
    alpha[0] = box_input_alpha(z[2] * cos(z[3]), dy->d_max[0], -1, pmin[0], pmax[0]);
    alpha[1] = box_input_alpha(z[2] * sin(z[3]), dy->d_max[1], -1, pmin[1], pmax[1]);
    alpha[2] = box_input_alpha(0.0, dy->a_max, +1, pmin[2], pmax[2]);
    if (dy->kind == HJO_CAR4D)
      alpha[3] = box_input_alpha(0.0, dy->w_max, +1, pmin[3], pmax[3]);
    else
      alpha[3] = box_input_alpha(0.0, fabs(z[2]) * tan(dy->steer_max) / dy->wheelbase, +1, pmin[3], pmax[3]);
    return;
  }
  int dir = dy->in_role == HJO_INPUT_MAXIMIZES ? 1 : -1;
  for (int d = 0; d < 4; ++d) {
    double b = dy->drift[d];
    if (!((dy->in_axes_mask >> d) & 1u)) {
      alpha[d] = fabs(b);
    } else if (dy->in_norm == HJO_BOX) {
      alpha[d] = box_input_alpha(b, dy->in_speed, dir, pmin[d], pmax[d]);
    } else {
      double gmin, gmax;
      ball_ratio_range(pmin, pmax, dy->in_axes_mask, d, &gmin, &gmax);
      double a = fabs(b + dir * dy->in_speed * gmax), c = fabs(b + dir * dy->in_speed * gmin);
      alpha[d] = a > c ? a : c;
    }
  }
}

/* max over the grid's nodes of hjo_alpha_box. */
void hjo_alpha_max_box(const hjo_grid *g, const hjo_dyn *dy, const double pmin[4], const double pmax[4],
                       double amax[4]) {
  for (int d = 0; d < 4; ++d) amax[d] = 0.0;
  int64_t np = hjo_num_points(g);
  for (int64_t p = 0; p < np; ++p) {
    int idx[4];
    double z[4], a[4];
    unravel(g, p, idx);
    for (int d = 0; d < 4; ++d) z[d] = hjo_node(g, d, idx[d]);
    hjo_alpha_box(dy, z, pmin, pmax, a);
    for (int d = 0; d < 4; ++d)
      if (a[d] > amax[d]) amax[d] = a[d];
  }
}

/* L = H(z, (p+ + p-)/2) + sum_d alpha_d (p+_d - p-_d) / 2 from the one-sided
 * derivatives of one node. */
static double lf_combine(const hjo_dyn *dy, const double z[4], const double alpha[4], const double pm[4],
                         const double pp[4]) {
  double pbar[4];
  for (int d = 0; d < 4; ++d) pbar[d] = (pp[d] + pm[d]) / 2.0;
  double diss = 0.0;
  for (int d = 0; d < 4; ++d) diss += alpha[d] * (pp[d] - pm[d]) / 2.0;
  return hamiltonian(dy, z, pbar) + diss;
}

static double rhs_at(const hjo_grid *g, const hjo_dyn *dy, int deriv, const double *V,
                     const int64_t st[4], int64_t p, const double *box) {
  int idx[4];
  double z[4], pm[4], pp[4], alpha[4];
  unravel(g, p, idx);
  for (int d = 0; d < 4; ++d) {
    z[d] = hjo_node(g, d, idx[d]);
    one_sided(g, deriv, V, st, p, idx, d, &pm[d], &pp[d]);
  }
  if (box)
    hjo_alpha_box(dy, z, box, box + 4, alpha);
  else
    alpha_at(dy, z, alpha);
  return lf_combine(dy, z, alpha, pm, pp);
}

/* L(V) at every node (outermost axis split across OpenMP threads; every
 * node is independent, so the result does not depend on the thread count). */
static void rhs_all(const hjo_grid *g, const hjo_dyn *dy, const hjo_scheme *sc, const double *V,
                    const double *box, double *L) {
  int64_t st[4];
  strides_of(g, st);
  int n0 = g->n[0];
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n0; ++i)
    for (int64_t q = 0; q < st[0]; ++q) {
      int64_t p = (int64_t)i * st[0] + q;
      L[p] = rhs_at(g, dy, sc->deriv, V, st, p, box);
    }
}

/* L(V); in the derivative-range mode alpha comes from V's own range. */
void hjo_rhs(const hjo_grid *g, const hjo_dyn *dy, const hjo_scheme *sc, const double *V,
             double *L) {
  double box[8];
  int range = sc->alpha_mode != HJO_ALPHA_STATE;
  if (range) hjo_deriv_range(g, sc, V, box, box + 4);
  rhs_all(g, dy, sc, V, range ? box : NULL, L);
}

/* ------------------------------------------------------------- steps --- */

/*
 * One full time step of length dt, in place on V.  work must hold 2 N
 * doubles.
 *   Euler (Algorithm 2):  V <- V + dt L(V).
 *   TVD-RK2 (textbook):    V1 = V + dt L(V);  V2 = V1 + dt L(V1);
 *                          V <- (V + V2) / 2.
 * Then, if the clamp is on, V <- min(V0, V) (once per full step).
 */
/* One step with alpha from `box` (the derivative range of V at the start of
 * the step; both TVD-RK2 stages use it) or the state bound (box NULL). */
static void step_with(const hjo_grid *g, const hjo_dyn *dy, const hjo_scheme *sc, const double *V0, double *V,
                      double dt, const double *box, double *work) {
  int64_t np = hjo_num_points(g);
  double *L = work, *V1 = work + np;
  rhs_all(g, dy, sc, V, box, L);
  if (sc->integrator == HJO_EULER) {
    for (int64_t p = 0; p < np; ++p) V[p] = V[p] + dt * L[p];
  } else {
    for (int64_t p = 0; p < np; ++p) V1[p] = V[p] + dt * L[p];
    rhs_all(g, dy, sc, V1, box, L);
    for (int64_t p = 0; p < np; ++p) {
      double v2 = V1[p] + dt * L[p];
      V[p] = (V[p] + v2) / 2.0;
    }
  }
  if (sc->clamp)
    for (int64_t p = 0; p < np; ++p)
      if (V0[p] < V[p]) V[p] = V0[p];
}

void hjo_step(const hjo_grid *g, const hjo_dyn *dy, const hjo_scheme *sc, const double *V0, double *V,
              double dt, double *work) {
  double box[8];
  int range = sc->alpha_mode != HJO_ALPHA_STATE;
  if (range) hjo_deriv_range(g, sc, V, box, box + 4);
  step_with(g, dy, sc, V0, V, dt, range ? box : NULL, work);
}

/* ------------------------- ENO choices as a binary32 evaluation takes them --- */

/*
 * The ENO choice is a comparison of two second differences, so where they are
 * close in magnitude the rounding of the arithmetic decides it.  To check a
 * binary32 (FP32) evaluation node by node, these functions take that decision
 * in binary32 as well: the window values rounded to binary32 (ghosts
 * extrapolated in binary32 by the rule of value_at), first and second
 * differences formed in binary32 in the same divided-difference form,
 * magnitudes compared, ties to the left.  Everything else -- the value of the
 * chosen second difference, the derivatives, H, the dissipation, the update --
 * stays binary64, as in the rest of this file.
 */

/* value_at in binary32: the node's value rounded to binary32, ghosts formed
 * from the rounded end values in binary32 arithmetic. */
static float value_at_f32(const hjo_grid *g, const double *V, const int64_t st[4], int64_t p, const int idx[4],
                          int d, int off) {
  int n = g->n[d];
  int i = idx[d] + off;
  int64_t base = p - (int64_t)idx[d] * st[d];
  if (i >= 0 && i < n) return (float)V[base + (int64_t)i * st[d]];
  if (is_periodic(g, d)) {
    i = ((i % n) + n) % n;
    return (float)V[base + (int64_t)i * st[d]];
  }
  if (i < 0) {
    float e = (float)V[base], nx = (float)V[base + st[d]];
    return e + (float)(-i) * (e - nx);
  }
  float e = (float)V[base + (int64_t)(n - 1) * st[d]], nx = (float)V[base + (int64_t)(n - 2) * st[d]];
  return e + (float)(i - (n - 1)) * (e - nx);
}

/*
 * One-sided derivatives along axis d with the ENO choices a binary32
 * evaluation takes.  A choice is "open" when tau > 0 and the binary32
 * magnitudes differ by at most tau * max(1, largest |window value|): inputs
 * that differ from these by that much rounding may take either side.  An open
 * choice returns both candidates: pm[0 .. *nm), pp[0 .. *np) hold one or two
 * values each.  First-order upwind has no choice.
 */
static void one_sided_f32dec(const hjo_grid *g, int deriv, const double *V, const int64_t st[4], int64_t p,
                             const int idx[4], int d, double tau, double pm[2], int *nm, double pp[2], int *np) {
  if (deriv == HJO_UPWIND1) {
    one_sided(g, deriv, V, st, p, idx, d, &pm[0], &pp[0]);
    *nm = *np = 1;
    return;
  }
  double h = hjo_spacing(g, d);
  double w[5];
  float f[5];
  for (int k = -2; k <= 2; ++k) {
    w[k + 2] = value_at(g, V, st, p, idx, d, k);
    f[k + 2] = value_at_f32(g, V, st, p, idx, d, k);
  }
  double d0 = w[1] - w[0], d1 = w[2] - w[1], d2 = w[3] - w[2], d3 = w[4] - w[3];
  double q_left = d1 - d0, q_mid = d2 - d1, q_right = d3 - d2;
  float e0 = f[1] - f[0], e1 = f[2] - f[1], e2 = f[3] - f[2], e3 = f[4] - f[3];
  float r_left = e1 - e0, r_mid = e2 - e1, r_right = e3 - e2;
  double scale = 1.0;
  for (int k = 0; k < 5; ++k)
    if (fabs((double)f[k]) > scale) scale = fabs((double)f[k]);
  double margin = tau * scale;
  /* p-: Q_{i-1} against Q_i */
  int left = fabsf(r_left) <= fabsf(r_mid);
  int open = tau > 0.0 && fabs((double)fabsf(r_left) - (double)fabsf(r_mid)) <= margin;
  pm[0] = d1 / h + (left ? q_left : q_mid) / (2.0 * h);
  *nm = 1;
  if (open) {
    pm[1] = d1 / h + (left ? q_mid : q_left) / (2.0 * h);
    *nm = 2;
  }
  /* p+: Q_i against Q_{i+1} */
  left = fabsf(r_mid) <= fabsf(r_right);
  open = tau > 0.0 && fabs((double)fabsf(r_mid) - (double)fabsf(r_right)) <= margin;
  pp[0] = d2 / h - (left ? q_mid : q_right) / (2.0 * h);
  *np = 1;
  if (open) {
    pp[1] = d2 / h - (left ? q_right : q_mid) / (2.0 * h);
    *np = 2;
  }
}

/*
 * Smallest and largest L(V) at one node over its open choices.  L is
 * nondecreasing in every p+_d and nonincreasing in every p-_d, because
 * alpha_d bounds |dH/dp_d| (dL/dp+_d = (dH/dp_d + alpha_d) / 2 >= 0,
 * dL/dp-_d = (dH/dp_d - alpha_d) / 2 <= 0): the smallest L takes on every
 * axis the smallest p+ and the largest p-, the largest L the reverse.
 */
static void rhs_interval_at(const hjo_grid *g, const hjo_dyn *dy, int deriv, const double *V, const int64_t st[4],
                            int64_t p, const double *box, double tau, double *Llo, double *Lhi) {
  int idx[4];
  double z[4], alpha[4], pm_lo[4], pm_hi[4], pp_lo[4], pp_hi[4];
  unravel(g, p, idx);
  for (int d = 0; d < 4; ++d) {
    double pm[2], pp[2];
    int nm, np;
    z[d] = hjo_node(g, d, idx[d]);
    one_sided_f32dec(g, deriv, V, st, p, idx, d, tau, pm, &nm, pp, &np);
    pm_lo[d] = pm_hi[d] = pm[0];
    if (nm == 2) {
      if (pm[1] < pm_lo[d]) pm_lo[d] = pm[1];
      if (pm[1] > pm_hi[d]) pm_hi[d] = pm[1];
    }
    pp_lo[d] = pp_hi[d] = pp[0];
    if (np == 2) {
      if (pp[1] < pp_lo[d]) pp_lo[d] = pp[1];
      if (pp[1] > pp_hi[d]) pp_hi[d] = pp[1];
    }
  }
  if (box)
    hjo_alpha_box(dy, z, box, box + 4, alpha);
  else
    alpha_at(dy, z, alpha);
  *Llo = lf_combine(dy, z, alpha, pm_hi, pp_lo);
  *Lhi = lf_combine(dy, z, alpha, pm_lo, pp_hi);
}

/*
 * One full step (as hjo_step, from V, leaving V unchanged) with the ENO
 * choices of a binary32 evaluation; lo[p], hi[p] = the smallest and largest
 * result at node p over its open choices (equal where none is open).  tau1
 * opens the choices of the first (or only) stage, taken on the caller's V;
 * tau2 those of the second TVD-RK2 stage, taken on V1 rounded to binary32 (a
 * binary32 evaluation stores V1 so, and its V1 differs from this one by its
 * rounding).  With TVD-RK2, tau1 must be 0: a first-stage choice left open
 * would give V1 an interval at a node whose neighbours' second-stage windows
 * hold it, and ENO2 is not monotone in its window.  Returns 0, -1 if memory
 * runs out, -2 for tau1 > 0 with TVD-RK2.
 */
int hjo_step_f32dec(const hjo_grid *g, const hjo_dyn *dy, const hjo_scheme *sc, const double *V0, const double *V,
                    double dt, double tau1, double tau2, double *lo, double *hi) {
  if (sc->integrator == HJO_TVD_RK2 && tau1 > 0.0) return -2;
  int64_t np = hjo_num_points(g);
  int64_t st[4];
  strides_of(g, st);
  double box[8];
  int range = sc->alpha_mode != HJO_ALPHA_STATE;
  if (range) hjo_deriv_range(g, sc, V, box, box + 4);
  const double *bx = range ? box : NULL;
  int n0 = g->n[0];
  if (sc->integrator == HJO_EULER) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n0; ++i)
      for (int64_t q = 0; q < st[0]; ++q) {
        int64_t p = (int64_t)i * st[0] + q;
        double a, b;
        rhs_interval_at(g, dy, sc->deriv, V, st, p, bx, tau1, &a, &b);
        lo[p] = V[p] + dt * a;
        hi[p] = V[p] + dt * b;
      }
  } else {
    double *V1 = (double *)malloc((size_t)np * sizeof(double));
    if (!V1) return -1;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n0; ++i)
      for (int64_t q = 0; q < st[0]; ++q) {
        int64_t p = (int64_t)i * st[0] + q;
        double a, b;
        rhs_interval_at(g, dy, sc->deriv, V, st, p, bx, 0.0, &a, &b);
        V1[p] = V[p] + dt * a;
      }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n0; ++i)
      for (int64_t q = 0; q < st[0]; ++q) {
        int64_t p = (int64_t)i * st[0] + q;
        double a, b;
        rhs_interval_at(g, dy, sc->deriv, V1, st, p, bx, tau2, &a, &b);
        double v2a = V1[p] + dt * a, v2b = V1[p] + dt * b;
        lo[p] = (V[p] + v2a) / 2.0;
        hi[p] = (V[p] + v2b) / 2.0;
      }
    free(V1);
  }
  if (sc->clamp)
    for (int64_t p = 0; p < np; ++p) {
      if (V0[p] < lo[p]) lo[p] = V0[p];
      if (V0[p] < hi[p]) hi[p] = V0[p];
    }
  return 0;
}

/*
 * Whole fixed-horizon solve: V := V0, then n = ceil(T / dt) steps with the
 * CFL step dt and a shortened last step.  Returns 0 on success, -1 if memory
 * runs out.
 */
int hjo_solve(const hjo_grid *g, const hjo_dyn *dy, const hjo_scheme *sc, const double *V0,
              double horizon, double *V, int64_t *n_steps, double *dt_out, double *dt_last_out) {
  int64_t np = hjo_num_points(g);
  if (sc->alpha_mode != HJO_ALPHA_STATE) {
    /* Algorithm 1: every step finds the derivative range, alpha and
     * dt = cfl / sum_d(alpha_d^max / dx_d); the step that would reach or pass
     * the horizon is shortened to end on it */
    double *work = (double *)malloc((size_t)np * 2 * sizeof(double));
    if (!work) return -1;
    memcpy(V, V0, (size_t)np * sizeof(double));
    double t = 0.0, first = 0.0, dtk = 0.0;
    int64_t n = 0;
    while (horizon > 0.0 && t < horizon) {
      double box[8], amax[4], S = 0.0;
      hjo_deriv_range(g, sc, V, box, box + 4);
      hjo_alpha_max_box(g, dy, box, box + 4, amax);
      for (int d = 0; d < 4; ++d) S += amax[d] / hjo_spacing(g, d);
      dtk = S == 0.0 ? horizon - t : sc->cfl / S;
      int last = t + dtk >= horizon;
      if (last) dtk = horizon - t;
      step_with(g, dy, sc, V0, V, dtk, box, work);
      if (n == 0) first = dtk;
      n += 1;
      if (last) break;
      t += dtk;
    }
    free(work);
    if (n_steps) *n_steps = n;
    if (dt_out) *dt_out = first;
    if (dt_last_out) *dt_last_out = n > 0 ? dtk : 0.0;
    return 0;
  }
  double dt = hjo_cfl_dt(g, dy, sc->cfl, horizon);
  int64_t n;
  double dt_last;
  hjo_schedule(dt, horizon, &n, &dt_last);
  double *work = (double *)malloc((size_t)np * 2 * sizeof(double));
  if (!work) return -1;
  memcpy(V, V0, (size_t)np * sizeof(double));
  for (int64_t k = 0; k < n; ++k) hjo_step(g, dy, sc, V0, V, k + 1 < n ? dt : dt_last, work);
  free(work);
  if (n_steps) *n_steps = n;
  if (dt_out) *dt_out = dt;
  if (dt_last_out) *dt_last_out = dt_last;
  return 0;
}

/*
 * Convergence-mode solve (Algorithms 1 and 2, last lines): V := V0, then
 * full steps of the CFL step dt while the change of the last step,
 * eps = max over nodes of |V_{t+1} - V_t|, is at or above `threshold`
 * (the printed test is inverted; the loop continues until the change falls
 * below the threshold), at most max_steps steps.  Returns 0, or -1 if memory
 * runs out; *n_steps = steps taken, *converged = 1 if eps < threshold
 * stopped it, *eps_last = eps of the last step.
 */
int hjo_solve_converge(const hjo_grid *g, const hjo_dyn *dy, const hjo_scheme *sc, const double *V0,
                       double threshold, int64_t max_steps, double *V, int64_t *n_steps, int32_t *converged,
                       double *eps_last, double *dt_out) {
  int64_t np = hjo_num_points(g);
  if (sc->alpha_mode != HJO_ALPHA_STATE) return -2;  /* a fixed step needs the state bound */
  double dt = hjo_cfl_dt(g, dy, sc->cfl, 1.0);
  double *work = (double *)malloc((size_t)np * 3 * sizeof(double));
  if (!work) return -1;
  double *prev = work + 2 * np;
  memcpy(V, V0, (size_t)np * sizeof(double));
  int64_t n = 0;
  int32_t conv = 0;
  double eps = 0.0;
  while (n < max_steps) {
    memcpy(prev, V, (size_t)np * sizeof(double));
    hjo_step(g, dy, sc, V0, V, dt, work);
    n += 1;
    eps = 0.0;
    for (int64_t i = 0; i < np; ++i) {
      double e = fabs(V[i] - prev[i]);
      if (e > eps || e != e) eps = e;
    }
    if (eps < threshold) {
      conv = 1;
      break;
    }
  }
  free(work);
  *n_steps = n;
  *converged = conv;
  *eps_last = eps;
  if (dt_out) *dt_out = dt;
  return 0;
}

/* ----------------------------------------------------- optimal control --- */

/* Gradient component d of V at a node: central difference inside, wrapped
 * on a periodic axis, one-sided at the ends of an open axis. */
static double node_grad(const hjo_grid *g, const double *V, const int64_t st[4], const int idx[4], int d) {
  int n = g->n[d], i = idx[d];
  double h = hjo_spacing(g, d);
  int64_t p = 0;
  for (int e = 0; e < 4; ++e) p += (int64_t)idx[e] * st[e];
  int64_t base = p - (int64_t)i * st[d];
  if (is_periodic(g, d)) {
    int im = i == 0 ? n - 1 : i - 1, ip = i == n - 1 ? 0 : i + 1;
    return (V[base + ip * st[d]] - V[base + im * st[d]]) / (2.0 * h);
  }
  if (i == 0) return (V[base + st[d]] - V[base]) / h;
  if (i == n - 1) return (V[base + (n - 1) * st[d]] - V[base + (n - 2) * st[d]]) / h;
  return (V[base + (i + 1) * st[d]] - V[base + (i - 1) * st[d]]) / (2.0 * h);
}

/*
 * Optimal control at arbitrary states (eq (9)): u = argmax_u grad V . f.
 * grad V and V at the state are multilinear interpolations over the 16
 * corners of the state's grid cell (of the nodal gradients above and of the
 * nodal values).  Cell: on an open axis the state is clamped to [lo, hi]
 * and i0 = min(floor((s - lo) / h), n - 2), weight (s - lo) / h - i0; on a
 * periodic axis t = (s - lo) / h reduced modulo n, i0 = floor(t),
 * i1 = (i0 + 1) mod n, weight t - i0.  Corners are visited with the theta
 * bit fastest; the weight of a corner is the product over x, y, v, theta (in
 * that order) of w_d or 1 - w_d.  Controls: a = +-a_max by the sign of p_v;
 * the car's w = +-w_max by the sign of p_theta, the steering car's
 * delta = +-steer_max by the sign of p_theta v (ties take +).  controls:
 * 2 per state; values: 1 per state; grads: 4 per state (may be NULL).
 * Returns -1 for dynamics without a control (the drift+input test model).
 */
int hjo_optimal_control(const hjo_grid *g, const hjo_dyn *dy, const double *V, const double *states, int64_t m,
                        double *controls, double *values, double *grads) {
  if (dy->kind != HJO_CAR4D && dy->kind != HJO_CAR4D_STEER) return -1;
  int64_t st[4];
  strides_of(g, st);
  for (int64_t q = 0; q < m; ++q) {
    const double *z = states + 4 * q;
    int i0[4], i1[4];
    double w[4];
    for (int d = 0; d < 4; ++d) {
      int n = g->n[d];
      double h = hjo_spacing(g, d);
      if (is_periodic(g, d)) {
        double t = (z[d] - g->lo[d]) / h;
        t = fmod(t, (double)n);
        if (t < 0.0) t += (double)n;
        int a = (int)floor(t);
        if (a >= n) a = n - 1;
        i0[d] = a;
        i1[d] = a + 1 == n ? 0 : a + 1;
        w[d] = t - (double)a;
      } else {
        double s = z[d] < g->lo[d] ? g->lo[d] : (z[d] > g->hi[d] ? g->hi[d] : z[d]);
        double t = (s - g->lo[d]) / h;
        int a = (int)floor(t);
        if (a > n - 2) a = n - 2;
        if (a < 0) a = 0;
        i0[d] = a;
        i1[d] = a + 1;
        w[d] = t - (double)a;
      }
    }
    double val = 0.0, p[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < 16; ++c) {
      int idx[4];
      double wt = 1.0;
      for (int d = 0; d < 4; ++d) {
        int bitd = (c >> (3 - d)) & 1;
        idx[d] = bitd ? i1[d] : i0[d];
        wt = wt * (bitd ? w[d] : 1.0 - w[d]);
      }
      int64_t off = 0;
      for (int d = 0; d < 4; ++d) off += (int64_t)idx[d] * st[d];
      val = val + wt * V[off];
      for (int d = 0; d < 4; ++d) p[d] = p[d] + wt * node_grad(g, V, st, idx, d);
    }
    controls[2 * q] = p[2] >= 0.0 ? dy->a_max : -dy->a_max;
    if (dy->kind == HJO_CAR4D)
      controls[2 * q + 1] = p[3] >= 0.0 ? dy->w_max : -dy->w_max;
    else
      controls[2 * q + 1] = p[3] * z[2] >= 0.0 ? dy->steer_max : -dy->steer_max;
    if (values) values[q] = val;
    if (grads)
      for (int d = 0; d < 4; ++d) grads[4 * q + d] = p[d];
  }
  return 0;
}

/* Thread count the OpenMP loops use (1 without OpenMP). */
int32_t hjo_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

void hjo_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
