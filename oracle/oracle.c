/*
 * oracle.c -- plain, slow CPU reference for the per-cell reaction burn.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP path: both read the same seeded input arrays and nothing else.
 *
 * What it computes (the paper, Sec. 2, "Arbitrary Network Generation": the
 * network's right-hand side and Jacobian are generated per network, and the
 * network is integrated with a VODE-class stiff integrator with self-heating;
 * Sec. 3 uses it cell by cell inside the hydrodynamics).  The paper writes out
 * neither the rate law nor the integrator, so this file fixes one reading and
 * states it next to each function:
 *
 *   y = (Y_1..Y_N, T),  rho fixed, log-rate multipliers p_r,
 *   lambda_r(T) = exp(a0 + a1/T + a2 T^-1/3 + a3 T^1/3 + a4 T + a5 T^5/3 + a6 ln T)
 *   R_r = e^{p_r} lambda_r rho^{n_r - 1} prod_j Y_j^{m_jr} / prod_j m_jr!
 *   dY_i/dt = sum_r nu_ir R_r,   dT/dt = (1/c_v) sum_r q_r R_r
 *
 * and integrates it with a variable-order (1..5) BDF in backward differences
 * with modified Newton and a dense partially pivoted LU of (I - c J), the
 * quasi-constant step-size scheme of Shampine & Reichelt (1997) with kappa = 0.
 *
 * Parity status: every function below is pinned by a CPU test (closed forms,
 * invariants, library routines, brute force) except the controller's choice
 * of step size and order, which has no outside reference: that part is
 * "parity unpinned" beyond the specification itself.
 *
 * Everything is IEEE double; build without fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_NMAX 64   /* max system size (species + 1) */
#define ORC_RMAX 512  /* max reactions */
#define ORC_KMAX 5    /* max BDF order */

/* Per-cell status codes. */
enum { ORC_OK = 0, ORC_MAX_STEPS = 1, ORC_STEP_UNDERFLOW = 2, ORC_NONFINITE = 3, ORC_BAD_INPUT = 4 };
/* Per-cell counters. */
enum { C_STEPS = 0, C_REJ_ERR, C_NEWTON_FAIL, C_RHS, C_JAC, C_LU, C_SOLVE, C_ORDER, C_COUNT };

typedef struct {
  int n_species, n_reactions;
  const int32_t *mass;      /* [N] */
  const int32_t *reactants; /* [R][3], -1 pad, repeats = multiplicity */
  const int32_t *products;  /* [R][3] */
  const double *coef;       /* [R][7] */
  const double *q;          /* [R] */
  double c_v;
  const double *screen;     /* [R] screening strengths h_r, or NULL */
  /* Test hook, 0 in every real run.  A nonzero value changes one rounding
   * step of the method (and nothing else) to measure how far two correct
   * implementations that round differently can drift apart:
   *   1  rate constants of reactions r = 0, 3, 6, ... taken one ulp up (a
   *      second exp / cbrt / log implementation);
   *   2  the species sums of the right-hand side taken in descending
   *      reaction order;
   *   3  the heat term multiplied by 1/c_v instead of divided by c_v. */
  int rounding_probe;
} orc_net;

typedef struct {
  double t_end, rtol, atol;
  int max_steps;
  /* Test hooks.  fixed_order = 0 runs the scheme as specified.  fixed_order
   * = k in 1..5 runs k-step BDF at the constant step fixed_h from the history
   * D_init (k+1 rows of backward differences), with no error test, no order or
   * step change, and Newton iterated to newton_tol_fixed. */
  int fixed_order;
  double fixed_h;
  const double *D_init;
  double newton_tol_fixed;
} orc_opts;

/* ------------------------------------------------------------------------ */
/* Rates (the ReacLib seven-parameter form)                                  */
/* ------------------------------------------------------------------------ */

/* lambda_r(T) and d ln lambda_r / dT for every reaction.  mult[r] = e^{p_r}
 * (or NULL for 1).  The seven basis functions are 1, 1/T, T^-1/3, T^1/3, T,
 * T^5/3, ln T. */
void orc_rates(const orc_net *net, double T, const double *log_mult, double *lam,
               double *dlnlam_dT) {
  double t13 = cbrt(T);
  double tm13 = 1.0 / t13;
  double t53 = T * t13 * t13;
  double lnT = log(T);
  double tinv = 1.0 / T;
  for (int r = 0; r < net->n_reactions; r++) {
    const double *a = net->coef + 7 * r;
    double expo = a[0] + a[1] * tinv + a[2] * tm13 + a[3] * t13 + a[4] * T + a[5] * t53 + a[6] * lnT;
    double l = exp(expo);
    if (net->rounding_probe == 1 && r % 3 == 0) l = nextafter(l, INFINITY);
    if (log_mult) l *= exp(log_mult[r]);
    lam[r] = l;
    if (dlnlam_dT) {
      /* d/dT of the exponent, term by term */
      dlnlam_dT[r] = -a[1] * tinv * tinv
                     - (1.0 / 3.0) * a[2] * tm13 * tinv
                     + (1.0 / 3.0) * a[3] * t13 * tinv
                     + a[4]
                     + (5.0 / 3.0) * a[5] * t13 * t13
                     + a[6] * tinv;
    }
  }
}

/* Number of reactant slots in use and 1 / prod(m_j!) for reaction r. */
static int reaction_order(const orc_net *net, int r, double *inv_fact) {
  const int32_t *s = net->reactants + 3 * r;
  int n = 0;
  for (int i = 0; i < 3; i++) n += (s[i] >= 0);
  /* multiplicities: count each distinct species */
  double f = 1.0;
  for (int i = 0; i < 3; i++) {
    if (s[i] < 0) continue;
    int first = 1, m = 0;
    for (int j = 0; j < i; j++) if (s[j] == s[i]) first = 0;
    if (!first) continue;
    for (int j = 0; j < 3; j++) m += (s[j] == s[i]);
    for (int j = 2; j <= m; j++) f *= (double)j;
  }
  *inv_fact = 1.0 / f;
  return n;
}

/* Synthetic screening (the network code applies plasma screening to its
 * rates, Sec. 2; no plasma data is used here): the rate of reaction r is
 * multiplied by F_r = exp(h_r G) with
 *   G(rho, T, Y) = sqrt(rho S) T^(-3/2),  S = 1 + sum_j A_j^2 Y_j,
 * a weak-screening-like dependence on density, temperature and composition.
 * Returns G and S. */
static double screen_G(const orc_net *net, double rho, const double *y, double *S_out) {
  int N = net->n_species;
  double S = 1.0;
  for (int j = 0; j < N; j++) S += (double)net->mass[j] * (double)net->mass[j] * y[j];
  *S_out = S;
  double T = y[N];
  return sqrt(rho * S) / (T * sqrt(T));
}

/* Reaction rates R_r at state y = (Y, T); lam receives the (screened) rate
 * constants. */
static void reaction_rates(const orc_net *net, double rho, const double *y, const double *log_mult,
                           double *R, double *lam, double *dlnlam) {
  int N = net->n_species;
  orc_rates(net, y[N], log_mult, lam, dlnlam);
  if (net->screen) {
    double S, G = screen_G(net, rho, y, &S);
    for (int r = 0; r < net->n_reactions; r++) lam[r] *= exp(net->screen[r] * G);
  }
  for (int r = 0; r < net->n_reactions; r++) {
    double inv_fact;
    int nr = reaction_order(net, r, &inv_fact);
    double v = lam[r] * inv_fact;
    for (int i = 1; i < nr; i++) v *= rho;
    const int32_t *s = net->reactants + 3 * r;
    for (int i = 0; i < 3; i++) if (s[i] >= 0) v *= y[s[i]];
    R[r] = v;
  }
}

/* Net stoichiometric coefficient nu_ir (products minus reactants). */
static int nu(const orc_net *net, int i, int r) {
  int v = 0;
  for (int s = 0; s < 3; s++) {
    v += (net->products[3 * r + s] == i);
    v -= (net->reactants[3 * r + s] == i);
  }
  return v;
}

/* Right-hand side f(y), n = N+1 entries. */
void orc_rhs(const orc_net *net, double rho, const double *y, const double *log_mult, double *f) {
  int N = net->n_species, Rn = net->n_reactions;
  double R[ORC_RMAX], lam[ORC_RMAX];
  reaction_rates(net, rho, y, log_mult, R, lam, NULL);
  for (int i = 0; i < N; i++) {
    double s = 0.0;
    for (int r = 0; r < Rn; r++) {
      int rr = net->rounding_probe == 2 ? Rn - 1 - r : r;
      int v = nu(net, i, rr);
      if (v) s += (double)v * R[rr];
    }
    f[i] = s;
  }
  double e = 0.0;
  for (int r = 0; r < Rn; r++) e += net->q[r] * R[r];
  f[N] = net->rounding_probe == 3 ? e * (1.0 / net->c_v) : e / net->c_v;
}

/* Analytic Jacobian J[i*n + j] = d f_i / d y_j (row-major, n = N+1).
 * dR_r/dY_j: derivative of the slot product, one term per slot holding j,
 * each term the product of the other slots (so Y_j = 0 is handled).
 * dR_r/dT = R_r * d ln lambda_r / dT.  With screening R_r also depends on
 * every Y_j and on T through G: dR_r/dY_j += R_r h_r dG/dY_j with
 * dG/dY_j = G A_j^2 / (2 S), and dR_r/dT += R_r h_r dG/dT, dG/dT = -3G/(2T). */
void orc_jac(const orc_net *net, double rho, const double *y, const double *log_mult, double *J) {
  int N = net->n_species, Rn = net->n_reactions, n = N + 1;
  double R[ORC_RMAX], lam[ORC_RMAX], dl[ORC_RMAX];
  reaction_rates(net, rho, y, log_mult, R, lam, dl);
  memset(J, 0, sizeof(double) * n * n);
  double G = 0.0, S = 1.0;
  if (net->screen) G = screen_G(net, rho, y, &S);
  for (int r = 0; r < Rn; r++) {
    double inv_fact;
    int nr = reaction_order(net, r, &inv_fact);
    double pre = lam[r] * inv_fact;
    for (int i = 1; i < nr; i++) pre *= rho;
    const int32_t *s = net->reactants + 3 * r;
    /* dR/dY_j for each distinct reactant species j */
    for (int a = 0; a < 3; a++) {
      if (s[a] < 0) continue;
      int j = s[a];
      double prod = pre;
      for (int b = 0; b < 3; b++) if (b != a && s[b] >= 0) prod *= y[s[b]];
      /* this slot's term of dR/dY_j */
      for (int i = 0; i < N; i++) {
        int v = nu(net, i, r);
        if (v) J[i * n + j] += (double)v * prod;
      }
      J[N * n + j] += net->q[r] * prod / net->c_v;
    }
    double dRdT = R[r] * dl[r];
    if (net->screen) {
      double u = net->screen[r] * R[r]; /* dR_r / dG */
      dRdT += u * (-1.5 * G / y[N]);
      for (int j = 0; j < N; j++) {
        double dRdY = u * G * (double)net->mass[j] * (double)net->mass[j] / (2.0 * S);
        for (int i = 0; i < N; i++) {
          int v = nu(net, i, r);
          if (v) J[i * n + j] += (double)v * dRdY;
        }
        J[N * n + j] += net->q[r] * dRdY / net->c_v;
      }
    }
    for (int i = 0; i < N; i++) {
      int v = nu(net, i, r);
      if (v) J[i * n + N] += (double)v * dRdT;
    }
    J[N * n + N] += net->q[r] * dRdT / net->c_v;
  }
}

/* ------------------------------------------------------------------------ */
/* Dense LU with partial pivoting                                            */
/* ------------------------------------------------------------------------ */

/* In-place LU of the n x n row-major matrix A with partial pivoting: at column
 * k the pivot is the first row p >= k with the largest |A[p][k]| (strict >
 * while scanning down, so ties go to the lowest row); rows k and p are swapped
 * in full.  piv[k] = p.  Returns 0, or k+1 if the pivot column k is all zero
 * (singular; A is then partially factored). */
int orc_lu_factor(int n, double *A, int *piv) {
  for (int k = 0; k < n; k++) {
    int p = k;
    double best = fabs(A[k * n + k]);
    for (int i = k + 1; i < n; i++) {
      double v = fabs(A[i * n + k]);
      if (v > best) { best = v; p = i; }
    }
    piv[k] = p;
    if (!(best > 0.0)) return k + 1;
    if (p != k) {
      for (int j = 0; j < n; j++) {
        double t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t;
      }
    }
    double d = A[k * n + k];
    for (int i = k + 1; i < n; i++) {
      double l = A[i * n + k] / d;
      A[i * n + k] = l;
      for (int j = k + 1; j < n; j++) A[i * n + j] -= l * A[k * n + j];
    }
  }
  return 0;
}

/* Solve A x = b with the factors from orc_lu_factor: apply the row swaps in
 * order, then forward substitution with the unit lower factor, then back
 * substitution with the upper factor.  b is overwritten with x. */
void orc_lu_solve(int n, const double *LU, const int *piv, double *b) {
  for (int k = 0; k < n; k++) {
    int p = piv[k];
    if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; }
  }
  for (int i = 0; i < n; i++) {
    double s = b[i];
    for (int j = 0; j < i; j++) s -= LU[i * n + j] * b[j];
    b[i] = s;
  }
  for (int i = n - 1; i >= 0; i--) {
    double s = b[i];
    for (int j = i + 1; j < n; j++) s -= LU[i * n + j] * b[j];
    b[i] = s / LU[i * n + i];
  }
}

/* ------------------------------------------------------------------------ */
/* BDF building blocks                                                       */
/* ------------------------------------------------------------------------ */

/* Weighted RMS norm sqrt((1/n) sum_i (v_i / s_i)^2), summed in ascending i. */
static double wrms(int n, const double *v, const double *s) {
  double acc = 0.0;
  for (int i = 0; i < n; i++) {
    double z = v[i] / s[i];
    acc += z * z;
  }
  return sqrt(acc / (double)n);
}

/* gamma_k = sum_{j=1..k} 1/j (gamma_0 = 0). */
static double bdf_gamma(int k) {
  double g = 0.0;
  for (int j = 1; j <= k; j++) g += 1.0 / (double)j;
  return g;
}

/* Generalised binomial C(s + j - 1, j) = s (s+1) ... (s+j-1) / j!. */
static double rising_binom(double s, int j) {
  double v = 1.0;
  for (int l = 0; l < j; l++) v *= (s + (double)l) / (double)(l + 1);
  return v;
}

/* Change the step size of the backward-difference history by the ratio rho_h.
 * Rows D_0..D_k hold the backward differences of the degree-k interpolant
 * p(t_n + s h) = sum_j D_j C(s + j - 1, j).  The new rows are obtained by
 * evaluating p at the new nodes s = -m rho_h (m = 0..k) and differencing
 * those values again: D'_a = sum_{m=0..a} (-1)^m C(a, m) p(-m rho_h).
 * D is stored row-major with n columns. */
void orc_rescale(int n, int k, double *D, double rho_h) {
  /* column by column: values of the interpolant at the new nodes, then
   * their backward differences */
  for (int i = 0; i < n; i++) {
    double v[ORC_KMAX + 1];
    for (int m = 0; m <= k; m++) {
      double s = -(double)m * rho_h;
      double acc = 0.0;
      for (int j = 0; j <= k; j++) acc += rising_binom(s, j) * D[j * n + i];
      v[m] = acc;
    }
    for (int a = 0; a <= k; a++) {
      double acc = 0.0;
      double binom = 1.0; /* C(a, m) */
      for (int m = 0; m <= a; m++) {
        double sign = (m % 2) ? -1.0 : 1.0;
        acc += sign * binom * v[m];
        binom = binom * (double)(a - m) / (double)(m + 1);
      }
      D[a * n + i] = acc;
    }
  }
}

static int all_finite(int n, const double *v) {
  for (int i = 0; i < n; i++) if (!isfinite(v[i])) return 0;
  return 1;
}

/* ------------------------------------------------------------------------ */
/* One cell                                                                  */
/* ------------------------------------------------------------------------ */

#define MIN_FACTOR 0.2
#define NEWTON_MAXIT 4
#define NEWTON_TOL 0.03

/* The frozen control decisions of a burn (what a sensitivity run replays):
 * the initial step size and, per accepted step, its BDF order, its step size
 * and the product of the history rescale ratios applied since the previous
 * accepted step (clamp onto t_end, rejections, Newton failures and the step
 * change chosen after the previous step).  Every rescale between two accepted
 * steps acts at the order of the later step. */
typedef struct {
  int cap;          /* capacity of the arrays */
  int n_steps;      /* accepted steps recorded */
  double h_init;    /* D_1 = h_init f(y0) */
  double *h;        /* [cap] */
  double *ratio;    /* [cap] */
  int32_t *order;   /* [cap] */
} orc_schedule;

static int burn_cell_impl(const orc_net *net, double rho, double *y_io, const double *log_mult,
                          const double *src, const orc_opts *o, int32_t *cnt,
                          orc_schedule *sch);
static void rhs_src(const orc_net *net, double rho, const double *y, const double *log_mult,
                    const double *src, double *f);

/* Initial step size (Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.4,
 * the starting-step algorithm for a method of order p = 1):
 *   s = atol + rtol |y0|, d0 = ||y0||, d1 = ||f(y0)|| (weighted RMS, scale s);
 *   h0 = 0.01 d0 / d1, or 1e-6 if d0 or d1 is below 1e-5; h0 <= t_end;
 *   one explicit Euler step y1 = y0 + h0 f(y0), d2 = ||f(y1) - f(y0)|| / h0;
 *   h1 = (0.01 / max(d1, d2))^(1/(p+1)), or max(1e-6, 1e-3 h0) when
 *   max(d1, d2) <= 1e-15 (and 1e-3 h0 when d2 is not finite);
 *   h = min(100 h0, h1, t_end).
 * f0 receives f(y0); *n_rhs counts the two evaluations.  Returns 0, or
 * ORC_NONFINITE when f(y0) is not finite (then *h_out is not set). */
static int initial_step(const orc_net *net, double rho, const double *y0, const double *log_mult,
                        const double *src, double t_end, double rtol, double atol, double *f0,
                        double *h_out, int *n_rhs) {
  const int n = net->n_species + 1;
  double s[ORC_NMAX], tmp[ORC_NMAX], f1[ORC_NMAX];
  rhs_src(net, rho, y0, log_mult, src, f0);
  (*n_rhs)++;
  if (!all_finite(n, f0)) return ORC_NONFINITE;
  for (int i = 0; i < n; i++) s[i] = atol + rtol * fabs(y0[i]);
  double d0 = wrms(n, y0, s), d1 = wrms(n, f0, s);
  double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
  if (h0 > t_end) h0 = t_end;
  for (int i = 0; i < n; i++) tmp[i] = y0[i] + h0 * f0[i];
  rhs_src(net, rho, tmp, log_mult, src, f1);
  (*n_rhs)++;
  for (int i = 0; i < n; i++) tmp[i] = f1[i] - f0[i];
  double d2 = wrms(n, tmp, s) / h0;
  double h1;
  if (!isfinite(d2)) {
    h1 = 1e-3 * h0;
  } else {
    double dm = d1 > d2 ? d1 : d2;
    if (dm <= 1e-15) {
      h1 = 1e-3 * h0;
      if (h1 < 1e-6) h1 = 1e-6;
    } else {
      h1 = sqrt(0.01 / dm);
    }
  }
  double h = 100.0 * h0;
  if (h1 < h) h = h1;
  if (t_end < h) h = t_end;
  *h_out = h;
  return ORC_OK;
}

/* Test entry: the initial step size the integrator takes for y0 (or -1 if
 * f(y0) is not finite). */
double orc_initial_step(const orc_net *net, double rho, const double *y0, const double *log_mult,
                        double t_end, double rtol, double atol) {
  double f0[ORC_NMAX], h = -1.0;
  int n_rhs = 0;
  if (initial_step(net, rho, y0, log_mult, NULL, t_end, rtol, atol, f0, &h, &n_rhs) != ORC_OK)
    return -1.0;
  return h;
}

/* Local error estimate of an order-k step (Shampine & Reichelt 1997, BDF
 * with kappa = 0): the corrector's total increment d = y_new - y_pred is
 * the (k+1)-th backward difference of the solution at the new point, and
 * the leading term of the local truncation error of BDF_k is C_k times it
 * with the error constant C_k = 1 / (k + 1).  The norm is the weighted RMS
 * with the scale s = atol + rtol max(|y_old|, |y_new|) componentwise, which
 * is returned in s_out (the order choice reuses it). */
double orc_error_norm(int n, int k, const double *d, const double *y_old, const double *y_new,
                      double rtol, double atol, double *s_out) {
  double tmp[ORC_NMAX];
  for (int i = 0; i < n; i++) {
    double a = fabs(y_old[i]), b = fabs(y_new[i]);
    s_out[i] = atol + rtol * (a > b ? a : b);
    tmp[i] = d[i] / (double)(k + 1);
  }
  return wrms(n, tmp, s_out);
}

/* Order and step-size choice after an accepted order-k step taken k+1 steps
 * after the last change (Shampine & Reichelt 1997).  After the history
 * update, D_k = grad^k y_{n+1} and D_{k+2} = grad^{k+2} y_{n+1}, so
 *   err_m = ||C_{k-1} D_k|| = ||D_k / k||          (order k-1, k > 1)
 *   err_p = ||C_{k+1} D_{k+2}|| = ||D_{k+2}/(k+2)||  (order k+1, k < 5)
 * estimate the local truncation errors the neighbouring orders would have
 * made, err (order k) is the step's own estimate, and each order q would
 * allow the step ratio err_q^(-1/(q+1)).  The order with the largest ratio
 * is taken (ties keep k, then prefer k-1); the new step ratio is
 * min(MAX_FACTOR, SAFETY * ratio).  dk, dk2: the rows D_k and D_{k+2};
 * s: the error test's scale.  Returns the new order; *factor the ratio. */
#define K_MAX 5
#define SAFETY 0.9
#define MAX_FACTOR 10.0
int orc_choose_order(int n, int k, double err, const double *dk, const double *dk2,
                     const double *s, double *factor) {
  double tmp[ORC_NMAX];
  double em = INFINITY, ep = INFINITY;
  if (k > 1) {
    for (int i = 0; i < n; i++) tmp[i] = dk[i] / (double)k;
    em = wrms(n, tmp, s);
  }
  if (k < K_MAX) {
    for (int i = 0; i < n; i++) tmp[i] = dk2[i] / (double)(k + 2);
    ep = wrms(n, tmp, s);
  }
  double fm = pow(em, -1.0 / (double)k);
  double f0 = pow(err, -1.0 / (double)(k + 1));
  double fp = pow(ep, -1.0 / (double)(k + 2));
  double best = f0;
  int dk_ = 0;
  if (fm > best) { best = fm; dk_ = -1; }
  if (fp > best) { best = fp; dk_ = 1; }
  double f = SAFETY * best;
  if (f > MAX_FACTOR) f = MAX_FACTOR;
  *factor = f;
  return k + dk_;
}

/* Integrate one cell from t = 0 to t_end.  y_io holds (Y, T) on entry and
 * the last accepted state on exit.  cnt receives the eight counters.  Returns
 * the status code. */
int orc_burn_cell(const orc_net *net, double rho, double *y_io, const double *log_mult,
                  const orc_opts *o, int32_t *cnt) {
  return burn_cell_impl(net, rho, y_io, log_mult, NULL, o, cnt, NULL);
}

/* orc_burn_cell that also returns the control decisions it took: the
 * initial step size, and per accepted step its order, its step size and the
 * product of the history rescale ratios since the previous accepted step
 * (arrays of cap entries; cap >= o->max_steps).  *n_rec receives the number
 * of recorded steps. */
int orc_burn_cell_sched(const orc_net *net, double rho, double *y_io, const double *log_mult,
                        const orc_opts *o, int32_t *cnt, double *h_init, double *h,
                        double *ratio, int32_t *order, int cap, int *n_rec) {
  orc_schedule sch;
  sch.cap = cap;
  sch.n_steps = 0;
  sch.h_init = 0.0;
  sch.h = h;
  sch.ratio = ratio;
  sch.order = order;
  int st = burn_cell_impl(net, rho, y_io, log_mult, NULL, o, cnt, &sch);
  *h_init = sch.h_init;
  *n_rec = sch.n_steps;
  return st;
}

/* Right-hand side plus a constant per-cell source term (src NULL: none).
 * The source is the advective forcing of the simplified-SDC coupling of
 * reactions and hydrodynamics that the network code supports (paper, Sec. 2):
 * over a hydro step the zone's reactions see the advective change of every
 * component as a constant rate, dy/dt = f(y) + A_adv. */
static void rhs_src(const orc_net *net, double rho, const double *y, const double *log_mult,
                    const double *src, double *f) {
  orc_rhs(net, rho, y, log_mult, f);
  if (src)
    for (int i = 0; i <= net->n_species; i++) f[i] = f[i] + src[i];
}

/* The integrator; when sch is not NULL the schedule is recorded (up to
 * sch->cap steps, which must be >= o->max_steps).  src: constant source
 * [n] or NULL. */
static int burn_cell_impl(const orc_net *net, double rho, double *y_io, const double *log_mult,
                          const double *src, const orc_opts *o, int32_t *cnt,
                          orc_schedule *sch) {
  const int N = net->n_species, n = N + 1;
  const double rtol = o->rtol, atol = o->atol, t_end = o->t_end;
  double D[(K_MAX + 3) * ORC_NMAX];
  double J[ORC_NMAX * ORC_NMAX], LU[ORC_NMAX * ORC_NMAX];
  int piv[ORC_NMAX];
  double y0[ORC_NMAX], f0[ORC_NMAX], f1[ORC_NMAX], s[ORC_NMAX], tmp[ORC_NMAX];
  double ypred[ORC_NMAX], psi[ORC_NMAX], d[ORC_NMAX], y[ORC_NMAX], F[ORC_NMAX], dy[ORC_NMAX];
  double s2[ORC_NMAX];
  for (int c = 0; c < C_COUNT; c++) cnt[c] = 0;

  /* Inputs: rho > 0, T > 0, everything finite. */
  if (!(rho > 0.0) || !isfinite(rho) || !(y_io[N] > 0.0) || !all_finite(n, y_io)) {
    return ORC_BAD_INPUT;
  }
  memcpy(y0, y_io, sizeof(double) * n);

  int k, n_eq = 0, jac_current, lu_valid = 0;
  double h, t = 0.0;

  if (o->fixed_order) {
    k = o->fixed_order;
    h = o->fixed_h;
    memset(D, 0, sizeof(D));
    memcpy(D, o->D_init, sizeof(double) * (k + 1) * n);
    orc_jac(net, rho, y0, log_mult, J);
    cnt[C_JAC]++;
    jac_current = 1;
  } else {
    /* Initial step (Hairer, Norsett & Wanner, vol. I, Sec. II.4, order 1). */
    int n_rhs = 0;
    int ist = initial_step(net, rho, y0, log_mult, src, t_end, rtol, atol, f0, &h, &n_rhs);
    cnt[C_RHS] += n_rhs;
    if (ist != ORC_OK) return ist;

    /* History: D_0 = y0, D_1 = h f0, the rest zero; order 1. */
    if (sch) { sch->h_init = h; sch->n_steps = 0; }
    k = 1;
    memset(D, 0, sizeof(D));
    for (int i = 0; i < n; i++) { D[i] = y0[i]; D[n + i] = h * f0[i]; }
    orc_jac(net, rho, y0, log_mult, J);
    cnt[C_JAC]++;
    if (!all_finite(n * n, J)) return ORC_NONFINITE;
    jac_current = 1;
  }

  int status = ORC_OK;
  double err = 0.0;
  double racc = 1.0; /* rescale ratios since the last accepted step */
  while (t < t_end) {
    if (cnt[C_STEPS] >= o->max_steps) { status = ORC_MAX_STEPS; break; }
    /* ---- one accepted step (with rejections and retries) ---- */
    int accepted = 0;
    double t_new = t;
    while (!accepted) {
      /* Step underflow: h below ten units in the last place of t (a
       * non-finite h counts too, so every cell terminates). */
      double ulp = nextafter(t, INFINITY) - t;
      if (!(h >= 10.0 * ulp)) { status = ORC_STEP_UNDERFLOW; break; }
      /* Land exactly on t_end. */
      t_new = t + h;
      if (t_new > t_end) {
        t_new = t_end;
        orc_rescale(n, k, D, (t_end - t) / h);
        racc *= (t_end - t) / h;
        h = t_end - t;
        n_eq = 0;
        lu_valid = 0;
      }
      /* Predictor, psi, Newton scale, c = h / gamma_k. */
      double gk = bdf_gamma(k);
      for (int i = 0; i < n; i++) {
        double a = 0.0;
        for (int j = 0; j <= k; j++) a += D[j * n + i];
        ypred[i] = a;
        double b = 0.0;
        for (int j = 1; j <= k; j++) b += bdf_gamma(j) * D[j * n + i];
        psi[i] = b / gk;
        s[i] = atol + rtol * fabs(ypred[i]);
      }
      double cc = h / gk;

      /* Modified Newton; on failure refresh a stale Jacobian once. */
      int converged = 0;
      for (;;) {
        int singular = 0;
        if (!lu_valid) {
          for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) LU[i * n + j] = (i == j ? 1.0 : 0.0) - cc * J[i * n + j];
          singular = orc_lu_factor(n, LU, piv);
          cnt[C_LU]++;
          lu_valid = 1;
        }
        if (!singular) {
          double tol = o->fixed_order ? o->newton_tol_fixed : NEWTON_TOL;
          int maxit = o->fixed_order ? 50 : NEWTON_MAXIT;
          double dprev = 0.0;
          for (int i = 0; i < n; i++) { d[i] = 0.0; y[i] = ypred[i]; }
          for (int it = 0; it < maxit; it++) {
            rhs_src(net, rho, y, log_mult, src, F);
            cnt[C_RHS]++;
            if (!all_finite(n, F)) break;
            for (int i = 0; i < n; i++) dy[i] = cc * F[i] - psi[i] - d[i];
            orc_lu_solve(n, LU, piv, dy);
            cnt[C_SOLVE]++;
            double dn = wrms(n, dy, s);
            if (!isfinite(dn)) break;
            double rate = 0.0;
            if (it > 0) {
              rate = dn / dprev;
              if (rate >= 1.0 || pow(rate, (double)(maxit - it)) / (1.0 - rate) * dn > tol) break;
            }
            for (int i = 0; i < n; i++) { y[i] += dy[i]; d[i] += dy[i]; }
            if (dn == 0.0 || (it > 0 && rate / (1.0 - rate) * dn < tol)) { converged = 1; break; }
            dprev = dn;
          }
        }
        /* A singular Newton matrix counts as a failed Newton attempt. */
        if (converged) break;
        cnt[C_NEWTON_FAIL]++;
        if (jac_current) break;
        orc_jac(net, rho, ypred, log_mult, J);
        cnt[C_JAC]++;
        jac_current = 1;
        lu_valid = 0;
      }
      if (!converged) {
        if (o->fixed_order) { status = ORC_STEP_UNDERFLOW; break; }
        /* Halve the step and retry. */
        h *= 0.5;
        orc_rescale(n, k, D, 0.5);
        racc *= 0.5;
        n_eq = 0;
        lu_valid = 0;
        continue;
      }

      /* Error test with scale atol + rtol * max(|y_n|, |y_new|). */
      err = orc_error_norm(n, k, d, D, y, rtol, atol, s2);
      if (!o->fixed_order && err > 1.0) {
        double factor = SAFETY * pow(err, -1.0 / (double)(k + 1));
        if (factor < MIN_FACTOR) factor = MIN_FACTOR;
        h *= factor;
        orc_rescale(n, k, D, factor);
        racc *= factor;
        n_eq = 0;
        lu_valid = 0;
        cnt[C_REJ_ERR]++;
        continue;
      }
      accepted = 1;
    }
    if (!accepted) break;

    /* Accept: update the differences. */
    t = t_new;
    for (int i = 0; i < n; i++) {
      D[(k + 2) * n + i] = d[i] - D[(k + 1) * n + i];
      D[(k + 1) * n + i] = d[i];
    }
    for (int j = k; j >= 0; j--)
      for (int i = 0; i < n; i++) D[j * n + i] += D[(j + 1) * n + i];
    jac_current = 0;
    n_eq++;
    if (sch && sch->n_steps < sch->cap) {
      sch->h[sch->n_steps] = h;
      sch->ratio[sch->n_steps] = racc;
      sch->order[sch->n_steps] = k;
      sch->n_steps++;
    }
    racc = 1.0;
    cnt[C_STEPS]++;
    if (o->fixed_order) continue;

    /* Order and step-size selection after k+1 steps at constant h. */
    if (n_eq >= k + 1) {
      double factor;
      k = orc_choose_order(n, k, err, D + k * n, D + (k + 2) * n, s2, &factor);
      h *= factor;
      orc_rescale(n, k, D, factor);
      racc *= factor;
      n_eq = 0;
      lu_valid = 0;
    }
  }
  cnt[C_ORDER] = k;
  memcpy(y_io, D, sizeof(double) * n);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Sensitivities with respect to the log-rate multipliers                    */
/* ------------------------------------------------------------------------ */

/* The question the paper asks of its networks is how the burn responds to
 * the individual rates (Sec. 1).  What is differentiated here is the burn
 * replayed on its own frozen schedule (orders, step sizes, rescale ratios of
 * the recorded run) with every corrector solved exactly, i.e. the discrete
 * map y0 -> y_end that the recorded run approximates to its Newton tolerance.
 * Its tangent-linear model gives S = d y_end / d p (forward sensitivities). */

#define ADJ_NEWTON_MAXIT 8
#define ADJ_NEWTON_TOL 1e-10

/* df/dp at y: Fp[i*R + r] = W_ir R_r, W = nu for a species row and q_r / c_v
 * for the temperature row (d R_r / d p_r = R_r). */
static void rhs_dlogmult(const orc_net *net, double rho, const double *y, const double *log_mult,
                         double *Fp) {
  int N = net->n_species, Rn = net->n_reactions;
  double R[ORC_RMAX], lam[ORC_RMAX];
  reaction_rates(net, rho, y, log_mult, R, lam, NULL);
  for (int i = 0; i < N; i++)
    for (int r = 0; r < Rn; r++) Fp[i * Rn + r] = (double)nu(net, i, r) * R[r];
  for (int r = 0; r < Rn; r++) Fp[N * Rn + r] = net->q[r] * R[r] / net->c_v;
}

/* Newton matrix I - c J(y) and its factors. */
static int newton_matrix(const orc_net *net, double rho, const double *y, const double *log_mult,
                         double c, double *J, double *LU, int *piv) {
  int n = net->n_species + 1;
  orc_jac(net, rho, y, log_mult, J);
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) LU[i * n + j] = (i == j ? 1.0 : 0.0) - c * J[i * n + j];
  return orc_lu_factor(n, LU, piv);
}

/* Replay schedule sch from y0 (y_io on entry) with exact correctors: full
 * Newton (Jacobian and factors at every iterate) from the predictor until the
 * weighted norm of the increment is <= ADJ_NEWTON_TOL, at most
 * ADJ_NEWTON_MAXIT iterations.  y_io receives y_end.  With S != NULL the
 * tangent-linear model is carried along and S (n x R, row-major) receives
 * d y_end / d p.  *n_unconv counts correctors that stopped at the iteration
 * limit.  Returns ORC_OK or ORC_NONFINITE (non-finite or singular corrector). */
int orc_replay_cell(const orc_net *net, double rho, double *y_io, const double *log_mult,
                    const orc_schedule *sch, double rtol, double atol, double *S, int *n_unconv) {
  const int N = net->n_species, n = N + 1, Rn = net->n_reactions;
  const int nc = n * Rn;
  double D[(K_MAX + 3) * ORC_NMAX];
  double J[ORC_NMAX * ORC_NMAX], LU[ORC_NMAX * ORC_NMAX];
  int piv[ORC_NMAX];
  double f0[ORC_NMAX], ypred[ORC_NMAX], psi[ORC_NMAX], s[ORC_NMAX], d[ORC_NMAX], y[ORC_NMAX];
  double F[ORC_NMAX], dy[ORC_NMAX];
  double *SD = NULL, *Fp = NULL, *Sy0 = NULL, *Spsi = NULL, *Sd = NULL;
  int status = ORC_OK;
  *n_unconv = 0;
  if (S) {
    SD = (double *)calloc((size_t)(K_MAX + 3) * nc, sizeof(double));
    Fp = (double *)malloc(sizeof(double) * nc);
    Sy0 = (double *)malloc(sizeof(double) * nc);
    Spsi = (double *)malloc(sizeof(double) * nc);
    Sd = (double *)malloc(sizeof(double) * nc);
  }
  memset(D, 0, sizeof(D));
  orc_rhs(net, rho, y_io, log_mult, f0);
  for (int i = 0; i < n; i++) { D[i] = y_io[i]; D[n + i] = sch->h_init * f0[i]; }
  if (S) {
    rhs_dlogmult(net, rho, y_io, log_mult, Fp);
    for (int q = 0; q < nc; q++) SD[nc + q] = sch->h_init * Fp[q];
  }
  for (int m = 0; m < sch->n_steps && status == ORC_OK; m++) {
    const int k = sch->order[m];
    const double h = sch->h[m], ratio = sch->ratio[m];
    if (ratio != 1.0) {
      orc_rescale(n, k, D, ratio);
      if (S) orc_rescale(nc, k, SD, ratio);
    }
    double gk = bdf_gamma(k);
    for (int i = 0; i < n; i++) {
      double a = 0.0;
      for (int j = 0; j <= k; j++) a += D[j * n + i];
      ypred[i] = a;
      double b = 0.0;
      for (int j = 1; j <= k; j++) b += bdf_gamma(j) * D[j * n + i];
      psi[i] = b / gk;
      s[i] = atol + rtol * fabs(ypred[i]);
      d[i] = 0.0;
      y[i] = ypred[i];
    }
    double cc = h / gk;
    int conv = 0;
    for (int it = 0; it < ADJ_NEWTON_MAXIT; it++) {
      orc_rhs(net, rho, y, log_mult, F);
      if (newton_matrix(net, rho, y, log_mult, cc, J, LU, piv)) { status = ORC_NONFINITE; break; }
      for (int i = 0; i < n; i++) dy[i] = cc * F[i] - psi[i] - d[i];
      orc_lu_solve(n, LU, piv, dy);
      double dn = wrms(n, dy, s);
      if (!isfinite(dn)) { status = ORC_NONFINITE; break; }
      for (int i = 0; i < n; i++) { y[i] += dy[i]; d[i] += dy[i]; }
      if (dn <= ADJ_NEWTON_TOL) { conv = 1; break; }
    }
    if (status != ORC_OK) break;
    if (!conv) (*n_unconv)++;
    if (S) {
      /* d' = M^-1 (c J y0' - psi' + c f_p), all at the corrected state */
      if (newton_matrix(net, rho, y, log_mult, cc, J, LU, piv)) { status = ORC_NONFINITE; break; }
      rhs_dlogmult(net, rho, y, log_mult, Fp);
      for (int q = 0; q < nc; q++) {
        double a = 0.0;
        for (int j = 0; j <= k; j++) a += SD[j * nc + q];
        Sy0[q] = a;
        double b = 0.0;
        for (int j = 1; j <= k; j++) b += bdf_gamma(j) * SD[j * nc + q];
        Spsi[q] = b / gk;
      }
      for (int r = 0; r < Rn; r++) {
        double col[ORC_NMAX];
        for (int i = 0; i < n; i++) {
          double jy = 0.0;
          for (int j = 0; j < n; j++) jy += J[i * n + j] * Sy0[j * Rn + r];
          col[i] = cc * jy - Spsi[i * Rn + r] + cc * Fp[i * Rn + r];
        }
        orc_lu_solve(n, LU, piv, col);
        for (int i = 0; i < n; i++) Sd[i * Rn + r] = col[i];
      }
    }
    /* the history update of an accepted step, for D and its tangent */
    for (int i = 0; i < n; i++) {
      D[(k + 2) * n + i] = d[i] - D[(k + 1) * n + i];
      D[(k + 1) * n + i] = d[i];
    }
    for (int j = k; j >= 0; j--)
      for (int i = 0; i < n; i++) D[j * n + i] += D[(j + 1) * n + i];
    if (S) {
      for (int q = 0; q < nc; q++) {
        SD[(k + 2) * nc + q] = Sd[q] - SD[(k + 1) * nc + q];
        SD[(k + 1) * nc + q] = Sd[q];
      }
      for (int j = k; j >= 0; j--)
        for (int q = 0; q < nc; q++) SD[j * nc + q] += SD[(j + 1) * nc + q];
    }
  }
  if (status == ORC_OK) {
    memcpy(y_io, D, sizeof(double) * n);
    if (S) memcpy(S, SD, sizeof(double) * nc);
  }
  free(SD); free(Fp); free(Sy0); free(Spsi); free(Sd);
  return status;
}

/* Per cell: burn with log_mult recording the schedule, then replay that
 * schedule from the same initial state with log_mult_replay (NULL: the same
 * multipliers), optionally with forward sensitivities.  Y, T receive the
 * replayed end state (the recorded run's state for a cell whose burn
 * failed); status the burn's status, or NONFINITE if the replay failed;
 * counters the burn's counters; S [C][n][R] (or NULL) the sensitivities,
 * zero for a failed cell; n_unconv [C] (or NULL) the correctors that hit the
 * iteration limit. */
int orc_sens_batch(const orc_net *net, int64_t n_cells, double *Y, const double *rho, double *T,
                   const double *log_mult, const double *log_mult_replay, const orc_opts *o,
                   int32_t *status, int32_t *counters, double *S, int32_t *n_unconv,
                   int n_threads) {
  int N = net->n_species, n = N + 1, Rn = net->n_reactions;
  if (N < 1 || n > ORC_NMAX || Rn < 1 || Rn > ORC_RMAX || n_cells < 0 || o->fixed_order)
    return -1;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t c = 0; c < n_cells; c++) {
    double y[ORC_NMAX], y0[ORC_NMAX];
    int32_t cnt[C_COUNT];
    orc_schedule sch;
    sch.cap = o->max_steps;
    sch.n_steps = 0;
    sch.h_init = 0.0;
    sch.h = (double *)malloc(sizeof(double) * sch.cap);
    sch.ratio = (double *)malloc(sizeof(double) * sch.cap);
    sch.order = (int32_t *)malloc(sizeof(int32_t) * sch.cap);
    for (int i = 0; i < N; i++) y[i] = Y[(int64_t)i * n_cells + c];
    y[N] = T[c];
    memcpy(y0, y, sizeof(double) * n);
    int st = burn_cell_impl(net, rho[c], y, log_mult, NULL, o, cnt, &sch);
    double *Sc = S ? S + (size_t)c * n * Rn : NULL;
    int unc = 0;
    if (st == ORC_OK) {
      int rs = orc_replay_cell(net, rho[c], y0, log_mult_replay ? log_mult_replay : log_mult,
                               &sch, o->rtol, o->atol, Sc, &unc);
      if (rs == ORC_OK) memcpy(y, y0, sizeof(double) * n);
      else st = rs;
    }
    if (Sc && st != ORC_OK) memset(Sc, 0, sizeof(double) * n * Rn);
    for (int i = 0; i < N; i++) Y[(int64_t)i * n_cells + c] = y[i];
    T[c] = y[N];
    if (status) status[c] = st;
    if (counters)
      for (int j = 0; j < C_COUNT; j++) counters[(int64_t)j * n_cells + c] = cnt[j];
    if (n_unconv) n_unconv[c] = unc;
    free(sch.h); free(sch.ratio); free(sch.order);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Batch driver (structure-of-arrays, like the GPU boundary)                 */
/* ------------------------------------------------------------------------ */

/* Burn n_cells independent cells.  Y is [N][C] (in/out), T is [C] (in/out),
 * rho is [C]; status [C] and counters [8][C] are outputs (either may be NULL).
 * n_threads <= 0 uses the OpenMP default.  Returns 0, or -1 on bad sizes. */
int orc_burn_batch(const orc_net *net, int64_t n_cells, double *Y, const double *rho, double *T,
                   const double *log_mult, const orc_opts *o, int32_t *status, int32_t *counters,
                   int n_threads) {
  int N = net->n_species;
  if (N < 1 || N + 1 > ORC_NMAX || net->n_reactions < 1 || net->n_reactions > ORC_RMAX ||
      n_cells < 0)
    return -1;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t c = 0; c < n_cells; c++) {
    double y[ORC_NMAX];
    int32_t cnt[C_COUNT];
    for (int i = 0; i < N; i++) y[i] = Y[(int64_t)i * n_cells + c];
    y[N] = T[c];
    int st = orc_burn_cell(net, rho[c], y, log_mult, o, cnt);
    for (int i = 0; i < N; i++) Y[(int64_t)i * n_cells + c] = y[i];
    T[c] = y[N];
    if (status) status[c] = st;
    if (counters)
      for (int j = 0; j < C_COUNT; j++) counters[(int64_t)j * n_cells + c] = cnt[j];
  }
  return 0;
}

/* orc_burn_batch with a constant per-cell source src [n][C] (rows: species,
 * then temperature). */
int orc_burn_batch_src(const orc_net *net, int64_t n_cells, double *Y, const double *rho,
                       double *T, const double *log_mult, const double *src, const orc_opts *o,
                       int32_t *status, int32_t *counters, int n_threads) {
  int N = net->n_species, n = N + 1;
  if (N < 1 || n > ORC_NMAX || net->n_reactions < 1 || net->n_reactions > ORC_RMAX ||
      n_cells < 0 || !src)
    return -1;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t c = 0; c < n_cells; c++) {
    double y[ORC_NMAX], sc[ORC_NMAX];
    int32_t cnt[C_COUNT];
    for (int i = 0; i < N; i++) y[i] = Y[(int64_t)i * n_cells + c];
    y[N] = T[c];
    for (int i = 0; i < n; i++) sc[i] = src[(int64_t)i * n_cells + c];
    int st = burn_cell_impl(net, rho[c], y, log_mult, sc, o, cnt, NULL);
    for (int i = 0; i < N; i++) Y[(int64_t)i * n_cells + c] = y[i];
    T[c] = y[N];
    if (status) status[c] = st;
    if (counters)
      for (int j = 0; j < C_COUNT; j++) counters[(int64_t)j * n_cells + c] = cnt[j];
  }
  return 0;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
