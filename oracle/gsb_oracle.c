/*
 * gsb_oracle.c -- plain CPU oracle for simulated bifurcation on the Ising problem.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference that
 * the GPU path is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header, table or
 * constant generator with the GPU library, and it never calls it.
 *
 * Source: Goto, Hidaka, Tatsumura, "Edge-of-chaos enhanced quantum-inspired algorithm
 * for combinatorial optimization" (arXiv 2508.17655).
 *   - Ising objective: eq. (1), Sec. II.
 *   - bSB update: eqs. (3)-(5) (symplectic Euler + perfectly inelastic walls), Sec. II.
 *   - linear schedule: eq. (6); individual control (GbSB): eq. (7), Sec. II.
 *   - dSB: J_ij x_j replaced by J_ij sgn(x_j) in eq. (3), Sec. VI.
 *   - order of the per-step arithmetic: y <- y + dy + Dy with dy = -p_i(t_{m+1}) x_i dt
 *     and Dy = c dt sum_j J_ij x_j; then x <- x + y(t_{m+1}) dt; then the wall
 *     (Fig. 2(a) caption, Sec. VI).
 *   - PXY arithmetic in 32-bit floating point (Fig. 2(a) caption, App. C).
 *   - initial conditions: x_i(0) uniform in (-0.1, 0.1), y_i(0) = 0 (App. A); the
 *     two-trajectory chaos start x = +-0.1 (Sec. IV).
 *   - normalised distance delta, eq. (8), and its trajectory pairs, Sec. IV.
 *   - forward and reverse derivatives of one continuous-product step, and the
 *     largest-Lyapunov-exponent estimate built on the forward one (not in the paper,
 *     which measures chaos with delta; the derivative is of eqs. (3)-(5), (7)).
 *
 * Two arithmetic modes:
 *   fp64 : every state variable and operation in binary64 (the "truth" used for
 *          error statements).
 *   fp32 : every state-update operation is one binary32 round-to-nearest-even
 *          operation in the order written below, no fused multiply-add (build with
 *          -ffp-contract=off).  The coupling sum is accumulated in binary64 in
 *          ascending j and rounded to binary32 once.  When J has entries in {0,+-1}
 *          and the operand is sign(x) or an E4M3 value, every partial sum is exactly
 *          representable, so the result is the exact product and any summation
 *          order gives the same bits.
 *
 * Readings where the paper is silent (listed with reasons in the design notes):
 *   - sgn(0) = +1 for spins and for the dSB operand.
 *   - wall: strict |x| > 1; x <- +-1 and y <- 0 in the same step.
 *   - A x^2 is evaluated as A * (x * x).
 *   - r_m = 1/(M - m) is evaluated in binary64 and rounded once (fp32 mode);
 *     c*dt likewise.
 *   - bSB/dSB are eq. (7) with A = 0, so they are bit-identical to GbSB/GdSB at A = 0.
 *   - counter-based SplitMix64 for the random initial conditions, one counter per
 *     (replica, stream, spin), so replica r's start does not depend on how many
 *     replicas run.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <fenv.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* variants */
enum { ORC_BSB = 0, ORC_DSB = 1, ORC_GBSB = 2, ORC_GDSB = 3 };
/* schedules */
enum { ORC_SCHED_LINEAR = 0, ORC_SCHED_CONSTANT = 1 };
/* operand forms for the continuous (bSB/GbSB) product */
enum { ORC_FORM_EXACT = 0, ORC_FORM_E4M3 = 1, ORC_FORM_BF16X2 = 2, ORC_FORM_FIX16 = 3 };
/* initial-condition modes */
enum { ORC_INIT_X = 0, ORC_INIT_XY = 1, ORC_INIT_PM01 = 2 };

/* ------------------------------------------------------------------------- */
/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014; public-domain C by S. Vigna). */
/* The k-th output (k >= 1) of the sequential generator seeded with s is       */
/* mix(s + k * golden_gamma).  Used here in that counter form.                 */
/* ------------------------------------------------------------------------- */
uint64_t orc_splitmix64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t orc_splitmix64_at(uint64_t seed, uint64_t k) { /* k-th output, k >= 1 */
  return orc_splitmix64_mix(seed + k * 0x9E3779B97F4A7C15ull);
}

/* uniform double in [0, 1) from the top 53 bits */
static double u01(uint64_t z) { return (double)(z >> 11) * 0x1.0p-53; }

/* Random initial state.  Counter for (replica r, stream s, spin i) is
 * (2 r + s) n + i, and the draw is output number counter + 1.
 *   mode X    : x ~ U(-0.1, 0.1) (stream 0), y = 0               (App. A)
 *   mode XY   : x and y ~ U(-0.1, 0.1) (streams 0 and 1)
 *   mode PM01 : x = +-0.1 with the sign from bit 63 of stream 0, y = 0 (Sec. IV)
 * x = (float)(-0.1 + 0.2 u), evaluated in binary64 and rounded once.           */
void orc_init_state(int n, int replicas, uint64_t seed, int mode, float* x, float* y) {
  for (int r = 0; r < replicas; ++r) {
    for (int i = 0; i < n; ++i) {
      uint64_t c0 = (uint64_t)(2 * (int64_t)r + 0) * (uint64_t)n + (uint64_t)i;
      uint64_t c1 = (uint64_t)(2 * (int64_t)r + 1) * (uint64_t)n + (uint64_t)i;
      uint64_t z0 = orc_splitmix64_at(seed, c0 + 1);
      float xv, yv = 0.0f;
      if (mode == ORC_INIT_PM01) {
        xv = (z0 >> 63) ? -0.1f : 0.1f;
      } else {
        double t = 0.2 * u01(z0);
        xv = (float)(-0.1 + t);
        if (mode == ORC_INIT_XY) {
          double t1 = 0.2 * u01(orc_splitmix64_at(seed, c1 + 1));
          yv = (float)(-0.1 + t1);
        }
      }
      x[(size_t)r * n + i] = xv;
      y[(size_t)r * n + i] = yv;
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Number formats, written from their definitions.                            */
/* ------------------------------------------------------------------------- */

/* OCP 8-bit floating point, E4M3 ("FN": no infinities, one NaN pattern S.1111.111):
 * 1 sign bit, 4 exponent bits with bias 7, 3 mantissa bits; normals 2^-6 .. 448,
 * subnormals k * 2^-9.  Conversion rounds to nearest, ties to even, and saturates
 * finite values beyond 448 to +-448. */
double orc_e4m3_round(double v) {
  if (isnan(v)) return v;
  double a = fabs(v);
  if (a == 0.0) return v;
  int e;
  frexp(a, &e);                 /* a = f 2^e, f in [0.5, 1): a in [2^(e-1), 2^e) */
  int E = e - 1;
  double q = (E < -6) ? ldexp(1.0, -9) : ldexp(1.0, E - 3); /* spacing of the grid */
  double k = nearbyint(a / q);  /* a/q is exact; default rounding is to nearest even */
  double r = k * q;
  if (r > 448.0) r = 448.0;
  return v < 0 ? -r : r;
}

uint8_t orc_e4m3_encode(double v) {
  if (isnan(v)) return 0x7F;
  uint8_t s = signbit(v) ? 0x80 : 0x00;
  double r = fabs(orc_e4m3_round(v));
  if (r == 0.0) return s;
  int e;
  frexp(r, &e);
  int E = e - 1;
  if (E < -6) return (uint8_t)(s | (uint8_t)(r / ldexp(1.0, -9)));
  int m = (int)((r / ldexp(1.0, E) - 1.0) * 8.0);
  return (uint8_t)(s | (uint8_t)(((E + 7) << 3) | m));
}

double orc_e4m3_decode(uint8_t b) {
  int s = b >> 7, E = (b >> 3) & 15, m = b & 7;
  double v;
  if (E == 15 && m == 7) return NAN;
  if (E == 0) v = ldexp((double)m, -9);
  else v = ldexp(1.0 + m / 8.0, E - 7);
  return s ? -v : v;
}

/* bfloat16: the top 16 bits of binary32, rounded to nearest, ties to even. */
float orc_bf16_round(float v) {
  if (isnan(v)) return v;
  uint32_t b;
  memcpy(&b, &v, 4);
  uint32_t lsb = (b >> 16) & 1u;
  b = (b + 0x7FFFu + lsb) & 0xFFFF0000u;
  float r;
  memcpy(&r, &b, 4);
  return r;
}

/* 16-bit fixed point with 14 fraction bits, round to nearest even (the precision
 * class of the paper's JX module, Fig. 2(a) caption); |x| <= 1 fits. */
double orc_fix16_round(double v) { return nearbyint(v * 16384.0) / 16384.0; }

/* ------------------------------------------------------------------------- */
/* Operand of the coupling product.                                           */
/* ------------------------------------------------------------------------- */
static int is_discrete(int variant) { return variant == ORC_DSB || variant == ORC_GDSB; }
static int has_control(int variant) { return variant == ORC_GBSB || variant == ORC_GDSB; }

static double operand(double x, int discrete, int form) {
  if (discrete) return x >= 0.0 ? 1.0 : -1.0; /* sgn with sgn(0) = +1 */
  switch (form) {
    case ORC_FORM_E4M3: return orc_e4m3_round(x);
    case ORC_FORM_BF16X2: {
      float xf = (float)x;
      float hi = orc_bf16_round(xf);
      float lo = orc_bf16_round(xf - hi); /* xf - hi is exact in binary32 */
      return (double)hi + (double)lo;
    }
    case ORC_FORM_FIX16: return orc_fix16_round(x);
    default: return x;
  }
}

/* ------------------------------------------------------------------------- */
/* Time stepping.                                                             */
/* One replica, steps m = m_begin .. m_end-1 of an M-step schedule.           */
/* State arrays: x, y, p of length n (this replica).                          */
/* ------------------------------------------------------------------------- */

/* fp64 mode */
static void run_replica_f64(const double* J, int n, int variant, int sched, int form,
                            double A, double dt, double c, int M, int m_begin, int m_end,
                            double* x, double* y, double* p, double* q, double* g,
                            double* traj /* nullable: [(m_end-m_begin)][n] x after each step */) {
  const double a = has_control(variant) ? A : 0.0;
  const int disc = is_discrete(variant);
  const double cdt = c * dt;
  for (int m = m_begin; m < m_end; ++m) {
    const double rm = (sched == ORC_SCHED_LINEAR) ? 1.0 / (double)(M - m) : 0.0;
    for (int j = 0; j < n; ++j) q[j] = operand(x[j], disc, form);
    for (int i = 0; i < n; ++i) { /* g_i = sum_j J_ij q_j, eq. (3) */
      double s = 0.0;
      const double* Ji = J + (size_t)i * n;
      for (int j = 0; j < n; ++j) s += Ji[j] * q[j];
      g[i] = s;
    }
    for (int i = 0; i < n; ++i) {
      double pn = p[i] - ((1.0 - a * (x[i] * x[i])) * p[i]) * rm; /* eq. (7) / (6) */
      double yn = (y[i] + (-(pn * x[i]) * dt)) + cdt * g[i];      /* eq. (3) */
      double xn = x[i] + yn * dt;                                 /* eq. (4) */
      if (fabs(xn) > 1.0) { xn = xn > 0 ? 1.0 : -1.0; yn = 0.0; } /* eq. (5) */
      p[i] = pn; y[i] = yn; x[i] = xn;
    }
    if (traj) memcpy(traj + (size_t)(m - m_begin) * n, x, sizeof(double) * (size_t)n);
  }
}

/* fp32 mode: each operation below is one binary32 operation (no contraction). */
static void run_replica_f32(const double* J, int n, int variant, int sched, int form,
                            double A, double dt, double c, int M, int m_begin, int m_end,
                            float* x, float* y, float* p, double* q, double* g,
                            float* traj) {
  const float a = has_control(variant) ? (float)A : 0.0f;
  const int disc = is_discrete(variant);
  const float dtf = (float)dt;
  const float cdt = (float)(c * dt);
  for (int m = m_begin; m < m_end; ++m) {
    const float rm = (sched == ORC_SCHED_LINEAR) ? (float)(1.0 / (double)(M - m)) : 0.0f;
    for (int j = 0; j < n; ++j) q[j] = operand((double)x[j], disc, form);
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      const double* Ji = J + (size_t)i * n;
      for (int j = 0; j < n; ++j) s += Ji[j] * q[j];
      g[i] = s;
    }
    for (int i = 0; i < n; ++i) {
      const float xi = x[i], yi = y[i], pi = p[i];
      const float gi = (float)g[i];
      float xx = xi * xi;
      float ax = a * xx;
      float f = 1.0f - ax;
      float fp = f * pi;
      float dp = fp * rm;
      float pn = pi - dp;           /* eq. (7) */
      float px = pn * xi;
      float pxdt = px * dtf;
      float y1 = yi - pxdt;         /* y + dy, dy = -p(t_{m+1}) x dt */
      float gy = cdt * gi;          /* Dy = c dt sum_j J_ij q_j */
      float yn = y1 + gy;           /* eq. (3) */
      float dx = yn * dtf;
      float xn = xi + dx;           /* eq. (4) */
      if (fabsf(xn) > 1.0f) { xn = xn > 0.0f ? 1.0f : -1.0f; yn = 0.0f; } /* eq. (5) */
      p[i] = pn; y[i] = yn; x[i] = xn;
    }
    if (traj) memcpy(traj + (size_t)(m - m_begin) * n, x, sizeof(float) * (size_t)n);
  }
}

/* Run `replicas` independent replicas (OpenMP over replicas only; the arithmetic of
 * each replica is exactly the sequential loop above).  J is n x n row-major.
 * x, y, p: [replicas][n], in/out.  traj (nullable): [replicas][m_end-m_begin][n].
 * Returns 0 on success, -1 on bad arguments. */
int orc_run_f64(const double* J, int n, int variant, int sched, int form, double A, double dt,
                double c, int M, int m_begin, int m_end, int replicas, double* x, double* y,
                double* p, double* traj) {
  if (n <= 0 || replicas <= 0 || M <= 0 || m_begin < 0 || m_end > M || m_begin > m_end) return -1;
  int bad = 0;
#pragma omp parallel for schedule(static)
  for (int r = 0; r < replicas; ++r) {
    double* q = (double*)malloc(sizeof(double) * (size_t)n);
    double* g = (double*)malloc(sizeof(double) * (size_t)n);
    if (!q || !g) { bad = 1; free(q); free(g); continue; }
    size_t o = (size_t)r * n;
    run_replica_f64(J, n, variant, sched, form, A, dt, c, M, m_begin, m_end, x + o, y + o, p + o,
                    q, g, traj ? traj + (size_t)r * (size_t)(m_end - m_begin) * n : NULL);
    free(q); free(g);
  }
  return bad ? -1 : 0;
}

int orc_run_f32(const double* J, int n, int variant, int sched, int form, double A, double dt,
                double c, int M, int m_begin, int m_end, int replicas, float* x, float* y,
                float* p, float* traj) {
  if (n <= 0 || replicas <= 0 || M <= 0 || m_begin < 0 || m_end > M || m_begin > m_end) return -1;
  int bad = 0;
#pragma omp parallel for schedule(static)
  for (int r = 0; r < replicas; ++r) {
    double* q = (double*)malloc(sizeof(double) * (size_t)n);
    double* g = (double*)malloc(sizeof(double) * (size_t)n);
    if (!q || !g) { bad = 1; free(q); free(g); continue; }
    size_t o = (size_t)r * n;
    run_replica_f32(J, n, variant, sched, form, A, dt, c, M, m_begin, m_end, x + o, y + o, p + o,
                    q, g, traj ? traj + (size_t)r * (size_t)(m_end - m_begin) * n : NULL);
    free(q); free(g);
  }
  return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------- */
/* Chaos diagnostics (Sec. IV) and the derivatives of one step.               */
/* ------------------------------------------------------------------------- */

/* Trajectory pairs of Sec. IV.  Pair k is replicas 2k and 2k+1:
 *   x1_i = +-0.1, the sign from bit 63 of the draw for counter (2k) n + i,
 *   x2_i = x1_i +- 2e-6, the sign from bit 63 of the draw for counter (2k+1) n + i,
 *   y = 0 for both (draw = SplitMix64 output number counter + 1, as in orc_init_state).
 * x2 is evaluated in binary64 from the binary32 x1 and rounded to binary32 once.  So x1
 * of pair k is x of replica k under ORC_INIT_PM01. */
void orc_init_pairs(int n, int pairs, uint64_t seed, float* x, float* y) {
  for (int k = 0; k < pairs; ++k) {
    for (int i = 0; i < n; ++i) {
      uint64_t c0 = (uint64_t)(2 * (int64_t)k + 0) * (uint64_t)n + (uint64_t)i;
      uint64_t c1 = (uint64_t)(2 * (int64_t)k + 1) * (uint64_t)n + (uint64_t)i;
      float x1 = (orc_splitmix64_at(seed, c0 + 1) >> 63) ? -0.1f : 0.1f;
      double d = (orc_splitmix64_at(seed, c1 + 1) >> 63) ? -2e-6 : 2e-6;
      x[(size_t)(2 * k) * n + i] = x1;
      x[(size_t)(2 * k + 1) * n + i] = (float)((double)x1 + d);
      y[(size_t)(2 * k) * n + i] = 0.0f;
      y[(size_t)(2 * k + 1) * n + i] = 0.0f;
    }
  }
}

/* Tangent (forward derivative) of the continuous-product step, binary64.  Variants bSB
 * and GbSB only: the sign product of dSB/GdSB is piecewise constant, its derivative 0.
 * Differentiating eqs. (7), (3), (4), (5) with f = 1 - A x^2 and r = r_m:
 *   p' = p (1 - f r)                     dp' = dp (1 - f r) + 2 A x dx p r
 *   y' = y - p' x dt + c dt (J x)        dy' = dy - (dp' x + p' dx) dt + c dt (J dx)
 *   x' = x + y' dt                       dx' = dx + dy' dt
 * and where the wall acts (|x'| > 1: x becomes the constant +-1, y becomes 0) the
 * component's dx' and dy' are 0.  One replica, steps m_begin .. m_end-1; the tangent
 * is first scaled to unit norm over (dx, dy, dp), then after every `renorm` steps (and
 * after the last) ln of its norm is added to *log_growth and it is scaled back to 1,
 * so *log_growth = ln(|v(t_end)| / |v(t_begin)|) of the unnormalised tangent. */
static void tangent_replica_f64(const double* J, int n, int sched, double a, double dt, double c, int M,
                                int m_begin, int m_end, int renorm, double* x, double* y, double* p,
                                double* dx, double* dy, double* dp, double* g, double* gd,
                                double* log_growth) {
  const double cdt = c * dt;
  double nrm = 0.0;
  for (int i = 0; i < n; ++i) nrm += dx[i] * dx[i] + dy[i] * dy[i] + dp[i] * dp[i];
  nrm = sqrt(nrm);
  for (int i = 0; i < n; ++i) { dx[i] /= nrm; dy[i] /= nrm; dp[i] /= nrm; }
  double lg = 0.0;
  for (int m = m_begin; m < m_end; ++m) {
    const double rm = (sched == ORC_SCHED_LINEAR) ? 1.0 / (double)(M - m) : 0.0;
    for (int i = 0; i < n; ++i) { /* the two products, J x and J dx, in ascending j */
      double s = 0.0, sd = 0.0;
      const double* Ji = J + (size_t)i * n;
      for (int j = 0; j < n; ++j) { s += Ji[j] * x[j]; sd += Ji[j] * dx[j]; }
      g[i] = s; gd[i] = sd;
    }
    for (int i = 0; i < n; ++i) {
      const double xi = x[i], yi = y[i], pi = p[i];
      const double f = 1.0 - a * (xi * xi);
      const double pn = pi - (f * pi) * rm;
      const double yn = (yi + (-(pn * xi) * dt)) + cdt * g[i];
      const double xn = xi + yn * dt;
      const double dpn = dp[i] * (1.0 - f * rm) + 2.0 * a * xi * dx[i] * pi * rm;
      const double dyn = dy[i] - (dpn * xi + pn * dx[i]) * dt + cdt * gd[i];
      const double dxn = dx[i] + dyn * dt;
      if (fabs(xn) > 1.0) {
        x[i] = xn > 0 ? 1.0 : -1.0; y[i] = 0.0; dx[i] = 0.0; dy[i] = 0.0;
      } else {
        x[i] = xn; y[i] = yn; dx[i] = dxn; dy[i] = dyn;
      }
      p[i] = pn; dp[i] = dpn;
    }
    const int done = m + 1 - m_begin;
    if ((renorm > 0 && done % renorm == 0) || m + 1 == m_end) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += dx[i] * dx[i] + dy[i] * dy[i] + dp[i] * dp[i];
      s = sqrt(s);
      lg += log(s);
      for (int i = 0; i < n; ++i) { dx[i] /= s; dy[i] /= s; dp[i] /= s; }
    }
  }
  *log_growth = lg;
}

/* Batch of replicas, arrays [replicas][n]; log_growth [replicas].  The largest
 * Lyapunov exponent estimate over the interval is log_growth / ((m_end - m_begin) dt).
 * Returns 0, or -1 on bad arguments (also for the sign-product variants). */
int orc_tangent_run_f64(const double* J, int n, int variant, int sched, double A, double dt, double c, int M,
                        int m_begin, int m_end, int renorm, int replicas, double* x, double* y, double* p,
                        double* dx, double* dy, double* dp, double* log_growth) {
  if (n <= 0 || replicas <= 0 || M <= 0 || m_begin < 0 || m_end > M || m_begin > m_end) return -1;
  if (is_discrete(variant)) return -1;
  const double a = has_control(variant) ? A : 0.0;
  int bad = 0;
#pragma omp parallel for schedule(static)
  for (int r = 0; r < replicas; ++r) {
    double* g = (double*)malloc(sizeof(double) * (size_t)n);
    double* gd = (double*)malloc(sizeof(double) * (size_t)n);
    if (!g || !gd) { bad = 1; free(g); free(gd); continue; }
    size_t o = (size_t)r * n;
    tangent_replica_f64(J, n, sched, a, dt, c, M, m_begin, m_end, renorm, x + o, y + o, p + o, dx + o, dy + o,
                        dp + o, g, gd, log_growth + r);
    free(g); free(gd);
  }
  return bad ? -1 : 0;
}

/* Adjoint (reverse derivative) of one continuous-product step, binary64, for one
 * replica at the step's input state (x, y, p) and r = r_m.  On entry (xb, yb, pb) are
 * the cotangents of the step's outputs; on return, of its inputs.  Transposing the
 * tangent above (J symmetric, so J^T w = J w) with k_i = [|x'_i| > 1]:
 *   w   = (1 - k) (yb + dt xb)
 *   pb' = pb - dt x w
 *   xb  = (1 - k) xb - dt p' w + c dt (J w) + 2 A x p r pb'
 *   yb  = w,  pb = pb' (1 - f r). */
int orc_adjoint_step_f64(const double* J, int n, int variant, double A, double dt, double c, double rm,
                         const double* x, const double* y, const double* p, double* xb, double* yb, double* pb) {
  if (n <= 0 || is_discrete(variant)) return -1;
  const double a = has_control(variant) ? A : 0.0;
  const double cdt = c * dt;
  double* g = (double*)malloc(sizeof(double) * (size_t)n);
  double* w = (double*)malloc(sizeof(double) * (size_t)n);
  double* gw = (double*)malloc(sizeof(double) * (size_t)n);
  if (!g || !w || !gw) { free(g); free(w); free(gw); return -1; }
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    const double* Ji = J + (size_t)i * n;
    for (int j = 0; j < n; ++j) s += Ji[j] * x[j];
    g[i] = s;
  }
  for (int i = 0; i < n; ++i) { /* forward step again, for p' and the wall mask */
    const double f = 1.0 - a * (x[i] * x[i]);
    const double pn = p[i] - (f * p[i]) * rm;
    const double yn = (y[i] + (-(pn * x[i]) * dt)) + cdt * g[i];
    const double xn = x[i] + yn * dt;
    const int k = fabs(xn) > 1.0;
    w[i] = k ? 0.0 : (yb[i] + dt * xb[i]);
    if (k) xb[i] = 0.0;
  }
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    const double* Ji = J + (size_t)i * n;
    for (int j = 0; j < n; ++j) s += Ji[j] * w[j];
    gw[i] = s;
  }
  for (int i = 0; i < n; ++i) {
    const double f = 1.0 - a * (x[i] * x[i]);
    const double pn = p[i] - (f * p[i]) * rm;
    const double pbn = pb[i] - dt * x[i] * w[i];
    xb[i] = xb[i] - dt * pn * w[i] + cdt * gw[i] + 2.0 * a * x[i] * p[i] * rm * pbn;
    yb[i] = w[i];
    pb[i] = pbn * (1.0 - f * rm);
  }
  free(g); free(w); free(gw);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Readout, energy, cut, best replica.                                        */
/* ------------------------------------------------------------------------- */

/* s_i = sgn(x_i), sgn(0) = +1 (x_i = sgn s_i, Sec. II). */
void orc_spins_f32(const float* x, int64_t count, int8_t* s) {
  for (int64_t k = 0; k < count; ++k) s[k] = x[k] >= 0.0f ? 1 : -1;
}
void orc_spins_f64(const double* x, int64_t count, int8_t* s) {
  for (int64_t k = 0; k < count; ++k) s[k] = x[k] >= 0.0 ? 1 : -1;
}

/* E = -1/2 sum_i sum_j J_ij s_i s_j, eq. (1); binary64, i-major, j ascending. */
void orc_energy(const double* J, int n, const int8_t* s, int replicas, double* E) {
#pragma omp parallel for schedule(static)
  for (int r = 0; r < replicas; ++r) {
    const int8_t* sr = s + (size_t)r * n;
    double acc = 0.0;
    for (int i = 0; i < n; ++i) {
      double hi = 0.0;
      for (int j = 0; j < n; ++j) hi += J[(size_t)i * n + j] * (double)sr[j];
      acc += (double)sr[i] * hi;
    }
    E[r] = -0.5 * acc;
  }
}

/* Cut value of the MAX-CUT instance with weights w = -J (Sec. III):
 * sum over i < j with s_i != s_j of w_ij, counted edge by edge. */
double orc_cut_direct(const double* J, int n, const int8_t* s) {
  double c = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (s[i] != s[j]) c += -J[(size_t)i * n + j];
  return c;
}

/* argmin_r E_r, ties to the smallest r. */
int orc_best(const double* E, int replicas) {
  int b = 0;
  for (int r = 1; r < replicas; ++r)
    if (E[r] < E[b]) b = r;
  return b;
}

/* Exhaustive ground state for n <= 24: spin n-1 fixed to +1 (E(s) = E(-s)),
 * the other n-1 spins enumerated in Gray-code order with local fields
 * h_i = sum_j J_ij s_j kept up to date.  Returns the minimum energy and one
 * minimiser in s_out. */
double orc_ground_state(const double* J, int n, int8_t* s_out) {
  if (n <= 0 || n > 24) return NAN;
  int8_t* s = (int8_t*)malloc((size_t)n);
  double* h = (double*)malloc(sizeof(double) * (size_t)n);
  for (int i = 0; i < n; ++i) s[i] = 1;
  double E = 0.0;
  for (int i = 0; i < n; ++i) {
    h[i] = 0.0;
    for (int j = 0; j < n; ++j) h[i] += J[(size_t)i * n + j] * s[j];
  }
  for (int i = 0; i < n; ++i) E += -0.5 * s[i] * h[i];
  double best = E;
  memcpy(s_out, s, (size_t)n);
  const uint64_t total = (n > 1) ? (1ull << (n - 1)) : 1ull;
  for (uint64_t k = 1; k < total; ++k) {
    int f = __builtin_ctzll(k); /* Gray code: flip bit f */
    /* flipping s_f changes E by 2 s_f h_f (J_ff = 0) */
    E += 2.0 * s[f] * h[f];
    for (int i = 0; i < n; ++i) h[i] -= 2.0 * J[(size_t)i * n + f] * s[f];
    s[f] = (int8_t)-s[f];
    if (E < best) { best = E; memcpy(s_out, s, (size_t)n); }
  }
  free(s); free(h);
  return best;
}

/* Normalised distance between two trajectories, eq. (8):
 * delta = sqrt( (1/(4N)) sum_i (x1_i - x2_i)^2 ). */
double orc_delta(const double* x1, const double* x2, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) { double d = x1[i] - x2[i]; s += d * d; }
  return sqrt(s / (4.0 * n));
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads the parallel loops over replicas use from here on (timing only; the results do
 * not depend on it: each replica is computed by one thread in a fixed order). */
void orc_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* Batch forms of the format conversions (for tests over many values). */
void orc_e4m3_round_array(const double* in, double* out, int64_t count) {
  for (int64_t k = 0; k < count; ++k) out[k] = orc_e4m3_round(in[k]);
}
void orc_e4m3_encode_array(const float* in, uint8_t* out, int64_t count) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < count; ++k) out[k] = orc_e4m3_encode((double)in[k]);
}
/* The value the coupling product of eq. (3) uses for each x: the operand form's rounding,
 * or the sign s(x) for the dSB/GdSB product (Sec. VI). */
void orc_operand_array(const float* in, double* out, int64_t count, int discrete, int form) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < count; ++k) out[k] = operand((double)in[k], discrete, form);
}
void orc_bf16_round_array(const float* in, float* out, int64_t count) {
  for (int64_t k = 0; k < count; ++k) out[k] = orc_bf16_round(in[k]);
}
