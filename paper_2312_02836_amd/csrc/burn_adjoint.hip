// burn_adjoint.hip -- sensitivities of the burn with respect to the
// per-reaction log-rate multipliers p_r (the rate-sensitivity question the
// paper raises in Sec. 1), by a discrete adjoint.
//
// What is differentiated: the burn replayed on its own frozen schedule.  A
// recording run (the production integrator, REC mode) stores for every
// accepted step its BDF order k_n, step size h_n and the product rho_n of the
// history rescale ratios applied since the previous accepted step (all at
// order k_n), plus the initial step size.  The replay then takes, per step,
//   D <- rescale(D, k_n, rho_n); y0 = sum_{j<=k} D_j;
//   psi = sum_{j=1..k} gamma_j D_j / gamma_k;  c = h_n / gamma_k;
//   d solves d + psi - c f(y0 + d; p) = 0 exactly (Newton to 1e-10);
//   D_{k+1} = d; D_j += D_{j+1} (j = k..0),
// starting from D_0 = y(0), D_1 = h_init f(y(0)), and y_end = D_0 (the
// integrator's row D_{k+2} only feeds error estimates, i.e. the frozen
// decisions, so it drops out of the map).  Every
// operation but the corrector is linear in D with schedule-only
// coefficients, so the reverse sweep is: transpose of the update, then the
// corrector's adjoint mu = M^-T lambda_d with M = I - c J(y_new),
// contributing c J^T mu to y0, -mu to psi and c R_r (sum_i W_ir mu_i) to
// dL/dp_r (W = nu for a species, q_r / c_v for temperature), then the
// transposes of the predictor, psi and the rescale.
//
// Memory: the schedule, a checkpoint of D every CK steps and the corrected
// states of one CK-step segment live in a caller-provided workspace.  When
// the workspace also holds a pool for the corrected states (its size from
// the recorded step counts), the replay keeps every cell's states there that
// fit, and the reverse sweep reads them; for the other cells it recomputes
// each segment forward from its checkpoint, keeping its corrected states, and
// walks it backwards.  Either way the states are the same doubles (the same
// replay arithmetic from the same history), so the gradients are too.
//
// Mapping: a cell per group of 32 lanes (two per wave) for systems of up to
// 32 components, else a whole wave; lane i of the group = component i.  The
// Newton matrix sits in LDS, one row per lane, and is factored there with
// row-position tracking; reactions are spread over the group's lanes.

#include "burn_body.h"

namespace bn {
namespace {

constexpr int CK = 16;          // accepted steps per checkpoint segment
constexpr int ADJ_MAXIT = 12;   // iterations of the exact corrector
constexpr double kChordRate = 0.1;  // slower contraction: a new Newton matrix
constexpr double ADJ_TOL = 1e-10;
constexpr int GR = 4;           // reactions per lane in the gradient (R <= 256)

// ---------------------------------------------------------------------------
// Recording run: the burn with the schedule recorder.

// The recording run on a persistent grid: lane groups take the next cell
// from a device queue counter (zeroed before the launch) as theirs finish.
template <int L, int S, int W>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W, W)))
burn_record_queue_kernel(BurnArgs a, unsigned long long *queue) {
  using SH = Shape<L, S>;
  extern __shared__ double smem[];
  load_tables(a.net, a.log_mult, smem);
  __syncthreads();
  const Tabs tb = tabs_at(smem, a.net.R);
  const int wave = threadIdx.x >> 6;
  double *wb = smem + tab_doubles_of(a.net.R) + (size_t)wave * SH::wave_doubles(a.net.n);
  run_cells<L, S, true, true>(a, tb, wb, 0, queue);
}

// ---------------------------------------------------------------------------
// Replay / adjoint kernel.
//
// A cell is owned by a group of G lanes, lane i of the group holding
// component i: G = 32 for systems of up to 32 components (two cells per
// wave), else 64.  The cells of a wave keep their own schedules: every loop
// over segments, steps and Newton iterations runs to the largest count among
// the wave's cells, each cell working only while its own count lasts, and
// every cross-lane operation stays inside a group.

// Per-cell LDS: six n-vectors (state, right-hand side accumulator, solve
// vector, J^T mu accumulator, reciprocal pivots, pivot rows), the Newton
// matrix (n rows, odd stride n | 1) and the gradient accumulators (R).  The
// corrected states of the segment being reversed live in the workspace
// (AdjArgs::seg).
__host__ __device__ inline int adj_vec_stride(int n) { return (n + 1) & ~1; }
__host__ __device__ inline size_t adj_cell_doubles(int n, int R) {
  return 6 * (size_t)adj_vec_stride(n) + (size_t)n * (size_t)(n | 1) + (size_t)((R + 1) & ~1);
}
__host__ __device__ inline int adj_group(int n) { return n <= 32 ? 32 : 64; }
__host__ __device__ inline size_t adj_wave_doubles(int n, int R) {
  return (size_t)(64 / adj_group(n)) * adj_cell_doubles(n, R);
}

// Component k (wave-uniform) of the lane's group.
template <int G>
__device__ __forceinline__ double group_read(double v, int k) {
  if constexpr (G == 64) {
    return readlane_f64(v, k);
  } else {
    static_assert(G == 32, "groups of 32 or 64 lanes");
    const double lo = readlane_f64(v, k), hi = readlane_f64(v, k + 32);
    return (threadIdx.x & 32) ? hi : lo;
  }
}

// Largest of a group-uniform value over the wave's groups.
template <int G>
__device__ __forceinline__ int wave_max_of_groups(int v) {
  int m = __builtin_amdgcn_readlane(v, 0);
  if constexpr (G == 32) {
    const int b = __builtin_amdgcn_readlane(v, 32);
    m = b > m ? b : m;
  }
  return m;
}

// Rate of reaction r at the state in ybuf (T-powers given) and its
// derivatives with respect to the reactant slots (g[0..2]) and T (g[3]).
struct TPow {
  double T, t13, tm13, t53, lnT, tinv;
};

__device__ __forceinline__ TPow tpow(double T) {
  TPow p;
  p.T = T;
  p.t13 = cbrt(T);
  p.tinv = 1.0 / T;
  p.tm13 = (p.t13 * p.t13) * p.tinv;  // T^(-1/3) = T^(2/3) / T
  p.t53 = T * p.t13 * p.t13;
  p.lnT = bn_log(T);
  return p;
}

__device__ __forceinline__ double rate_and_slots(const Tabs &tb, int r, const TPow &tp,
                                                 const double *ybuf, double rho, bool want_g,
                                                 double g[4]) {
  const Coef c = coef_of(tb.rtab, r);
  const double expo = c[0] + c[1] * tp.tinv + c[2] * tp.tm13 + c[3] * tp.t13 + c[4] * tp.T +
                      c[5] * tp.t53 + c[6] * tp.lnT;
  const int4 spv = *reinterpret_cast<const int4 *>(tb.rsp + 4 * r);
  const int sp[4] = {spv.x, spv.y, spv.z, spv.w};
  // unconditional slot loads (an absent slot reads entry 0 and stands for 1)
  const double fa = ybuf[sp[0] < 0 ? 0 : sp[0]];
  const double fb = ybuf[sp[1] < 0 ? 0 : sp[1]];
  const double fc = ybuf[sp[2] < 0 ? 0 : sp[2]];
  double pre = exp(expo) * tb.emult[r] * c[7];
  // rho^(n_r - 1) for n_r <= 3 reactants
  if (sp[3] >= 2) pre *= rho;
  if (sp[3] >= 3) pre *= rho;
  const double ya = sp[0] >= 0 ? fa : 1.0;
  const double yb = sp[1] >= 0 ? fb : 1.0;
  const double yc = sp[2] >= 0 ? fc : 1.0;
  double full = pre;
  if (sp[0] >= 0) full *= ya;
  if (sp[1] >= 0) full *= yb;
  if (sp[2] >= 0) full *= yc;
  if (want_g) {
    const double dl = -c[1] * tp.tinv * tp.tinv - (1.0 / 3.0) * c[2] * tp.tm13 * tp.tinv +
                      (1.0 / 3.0) * c[3] * tp.t13 * tp.tinv + c[4] +
                      (5.0 / 3.0) * c[5] * tp.t13 * tp.t13 + c[6] * tp.tinv;
    g[0] = pre;
    g[1] = pre;
    g[2] = pre;
    g[3] = full * dl;
    if (sp[1] >= 0) g[0] *= yb;
    if (sp[2] >= 0) g[0] *= yc;
    if (sp[0] >= 0) g[1] *= ya;
    if (sp[2] >= 0) g[1] *= yc;
    if (sp[0] >= 0) g[2] *= ya;
    if (sp[1] >= 0) g[2] *= yb;
  }
  return full;
}

__device__ __forceinline__ void lds_add(double *p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// BACKWARD = false: replay from y(0), write the checkpoints, the end state
// and E.  BACKWARD = true: reverse sweep.  W is the waves per SIMD the
// registers are budgeted for (3 when the LDS lets three waves per SIMD
// reside, else 2); G the lanes per cell.  POOL (reverse sweep): the
// instance for the cells whose corrected states are in the pool, without
// the segment recomputation (its registers alone; the other cells rest).
template <bool BACKWARD, int W, int G, bool POOL = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W, W)))
adjoint_kernel(AdjArgs a) {
  constexpr int CPW = 64 / G;   // cells per wave
  extern __shared__ double smem[];
  load_tables(a.net, a.log_mult, smem);
  __syncthreads();
  const Tabs tb = tabs_at(smem, a.net.R);
  const NetTables &nt = a.net;
  const int N = nt.N, R = nt.R, n = nt.n;
  const int ne = nt.max_ent;  // entries per reaction, padded (ent_of)
  const int MS = n | 1, VS = adj_vec_stride(n);
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int cs = lane / G;  // the lane's cell slot in the wave
  const int i = lane % G;   // the lane's component
  const int64_t C = a.n_cells;
  const int64_t first = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * CPW;
  if (first >= C) return;  // whole wave: no later workgroup barrier
  const bool valid = first + cs < C;
  // the cell at this position (an empty slot reads a real cell)
  const int64_t p = valid ? first + cs : C - 1;
  const int64_t cell = a.order ? (int64_t)a.order[p] : p;

  double *wb = smem + tab_doubles_of(R) + (size_t)wave * adj_wave_doubles(n, R) +
               (size_t)cs * adj_cell_doubles(n, R);
  double *ybuf = wb;
  double *facc = wb + VS;
  double *vbuf = wb + 2 * VS;
  double *jout = wb + 3 * VS;
  double *dinvp = wb + 4 * VS;
  int *prow = reinterpret_cast<int *>(wb + 5 * VS);
  double *M = wb + 6 * VS;
  double *grl = M + (size_t)n * MS;  // gradient accumulators, reaction r on lane r % G

  const bool own = i < n;  // lane owns component i
  const double rho = a.rho[cell];
  const double *blk = a.sched + cell * a.sched_stride;
  const int n_rec = (int)blk[0];
  const double *sh = blk + 2;
  const double *sr = blk + 2 + a.sched_cap;
  const int32_t *so = reinterpret_cast<const int32_t *>(blk + 2 + 2 * (int64_t)a.sched_cap);
  double *ck = a.ckpt + (size_t)cell * a.n_ckpt * 7 * n;
  // this cell's corrected states in the pool ([step][n]), or none
  const int64_t so_off = a.soff ? a.soff[cell] : -1;
  const bool has_states = so_off >= 0 && valid;
  double *yst = has_states ? a.states + so_off : nullptr;

  // every slot starts with a valid pivot order and a finite state, so that
  // the group operations a resting cell takes part in stay in bounds
  if (own) {
    prow[i] = i;
    dinvp[i] = 1.0;
    ybuf[i] = 1.0;
  }

  // a cell of the other part of a split reverse sweep rests here
  const bool skip = BACKWARD && ((a.part == 1 && !has_states) || (a.part == 2 && has_states));
  // a failed recording run (or, backward, a failed replay): no replay
  const int st_in = a.status[cell];
  const bool dead = !valid || n_rec < 0 || st_in != ST_OK || skip;
  if (dead && valid && !skip) {
    if constexpr (BACKWARD) {
      for (int r = i; r < R; r += G) a.grad[(int64_t)r * C + cell] = 0.0;
    } else {
      if (i == 0) {
        a.Eout[cell] = (a.Tout[cell] - a.T0[cell]) / nt.inv_cv;
        if (a.iters) a.iters[cell] = a.iters[C + cell] = 0;
      }
    }
  }
  // a reverse-sweep wave with no live cell has nothing more to write
  if constexpr (BACKWARD) {
    if (__ballot(!dead) == 0) return;
  }
  const int nst = dead ? 0 : n_rec;  // this cell's accepted steps

  // initial state
  double y0v = 0.0;
  if (own) y0v = (i < N) ? a.Y0[(int64_t)i * C + cell] : a.T0[cell];

  // ---- group building blocks ----
  // F = f(y) (component i) for cells with want_f; the Newton matrix I - cJ(y)
  // into M for cells with want_m.  y is taken from ybuf.  Returns 1 if
  // everything evaluated is finite.
  auto eval_f_m = [&](double c, bool want_f, bool want_m, double &f_out) -> int {
    if (want_f && own) facc[i] = 0.0;
    if (want_m && own)
      for (int j = 0; j < n; ++j) M[i * MS + j] = (i == j) ? 1.0 : 0.0;
    wave_lds_sync();
    const TPow tp = tpow(ybuf[N]);
    double heat = 0.0;
    int bad = 0;
    for (int r = i; r < R; r += G) {
      double g[4];
      const double v = rate_and_slots(tb, r, tp, ybuf, rho, want_m, g);
      const int4 *ro = reinterpret_cast<const int4 *>(tb.rout + 8 * r);
      const int4 r0 = ro[0], r1 = ro[1];
      if (want_f) {
        heat += tb.q[r] * v;
        Unroll<6>::run([&]<int E>() __attribute__((always_inline)) {
          if (E < ne) {
            const Ent en = ent_of<E>(r0, r1);
            lds_add(&facc[en.sp], en.w * v);
          }
        });
      }
      if (want_m) {
        const int *sp = tb.rsp + 4 * r;
        const double qc = tb.qcv[r];
        for (int s = 0; s < 4; ++s) {
          const int col = (s < 3) ? sp[s] : N;
          if (col < 0) continue;
          if (!isfinite(g[s])) bad = 1;
          const double val = -c * g[s];
          Unroll<6>::run([&]<int E>() __attribute__((always_inline)) {
            if (E < ne) {
              const Ent en = ent_of<E>(r0, r1);
              lds_add(&M[en.sp * MS + col], en.w * val);
            }
          });
          lds_add(&M[N * MS + col], qc * val);
        }
      }
    }
    heat = gsum<G>(heat);
    wave_lds_sync();
    f_out = 0.0;
    if (want_f && own) f_out = (i < N) ? facc[i] : heat * nt.inv_cv;
    if (own && !isfinite(f_out)) bad = 1;
    return !gor<G>(bad);
  };

  // LU of M in place for cells with do_f (rows stay put; prow[p] = physical
  // row at position p, dinvp[p] = 1/U_pp).  Every lane takes part in the
  // pivot searches.  Returns 1 if nonsingular.
  auto factor = [&](bool do_f) -> int {
    int pos = i;
    int sing = 0;
    double fdinv = 1.0;
    double *Mrow = M + (own ? i : 0) * MS;
    for (int K = 0; K < n; ++K) {
      double v = -2.0;
      int nan_k = 0;
      const bool cand = own && pos >= K;
      if (cand) {
        v = fabs(Mrow[K]);
        if (v != v) {
          if (pos == K) nan_k = 1;
          v = -1.0;
        }
      }
      int key = cand ? ((pos << 8) | i) : 0x7fffffff;
      gargmax_key<G>(v, key);
      const int bp = key >> 8, prow_i = key & 255;
      nan_k = gor<G>(nan_k);
      if (!(v > 0.0) || nan_k) sing = 1;
      if (own) {
        if (pos == K) pos = bp;
        else if (pos == bp) pos = K;
      }
      const double *P = M + prow_i * MS;
      const double rinv = 1.0 / P[K];
      if (own && pos == K) fdinv = rinv;
      if (do_f && own && pos > K) {
        const double l = Mrow[K] * rinv;
        Mrow[K] = l;
        // whole chunks of 4 columns (loads issued together), then the rest
        int j0 = K + 1;
        for (; j0 + 4 <= n; j0 += 4) {
          double x[4], y[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            x[u] = Mrow[j0 + u];
            y[u] = P[j0 + u];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            x[u] -= l * y[u];
            Mrow[j0 + u] = x[u];
          }
        }
        for (; j0 < n; ++j0) Mrow[j0] -= l * P[j0];
      }
      wave_lds_sync();
    }
    if (do_f && own) {
      prow[pos] = i;
      dinvp[pos] = fdinv;
    }
    wave_lds_sync();
    return !sing;
  };

  // x = M^-1 b (b, x: component i)
  auto solve = [&](double b) -> double {
    if (own) vbuf[i] = b;
    wave_lds_sync();
    const int pr = own ? prow[i] : 0;  // lane works on position i
    double z = own ? vbuf[pr] : 0.0;
    const double *Lrow = M + pr * MS;
    for (int K = 0; K < n; ++K) {
      const double zk = group_read<G>(z, K);
      if (own && i > K) z -= Lrow[K] * zk;
    }
    const double dv = own ? dinvp[i] : 1.0;
    for (int K = n - 1; K >= 0; --K) {
      const double xk = group_read<G>(z * dv, K);
      if (i == K) z = xk;
      if (own && i < K) z -= Lrow[K] * xk;
    }
    wave_lds_sync();
    return z;  // position i = column i
  };

  // y = M^-T c (c, y: component i)
  auto solve_t = [&](double cv) -> double {
    // U^T w = c over positions (lane p holds w_p), then L^T v = w, y = P^T v
    double w = own ? cv : 0.0;
    double acc = 0.0;
    for (int K = 0; K < n; ++K) {
      const double wk = group_read<G>((w - acc) * (own ? dinvp[i] : 1.0), K);
      if (i == K) w = wk;
      const int rk = prow[K];
      if (own && i > K) acc += M[rk * MS + i] * wk;
    }
    double v = w;
    for (int K = n - 1; K >= 0; --K) {
      const double vk = group_read<G>(v, K);
      const int rk = prow[K];
      if (own && i < K) v -= M[rk * MS + i] * vk;
    }
    if (own) vbuf[prow[i]] = v;
    wave_lds_sync();
    const double y = own ? vbuf[i] : 0.0;
    wave_lds_sync();
    return y;
  };

  auto wrms = [&](double v, double inv) -> double {
    const double z = own ? v * inv : 0.0;
    return sqrt(gsum<G>(z * z) / (double)n);
  };

  // history rows of this lane's component
  double D[DROWS];
#pragma unroll
  for (int j = 0; j < DROWS; ++j) D[j] = 0.0;

  auto rescale_fwd = [&](int k, double rh) {
    double v[KMAX + 1];
#pragma unroll
    for (int m = 0; m <= KMAX; ++m) {
      const double x = (double)m * rh;
      double rb = 1.0, acc = D[0];
#pragma unroll
      for (int b = 1; b <= KMAX; ++b) {
        rb *= ((double)(b - 1) - x) * (1.0 / (double)b);
        if (b <= k) acc += rb * D[b];
      }
      v[m] = acc;
    }
#pragma unroll
    for (int aa = 0; aa <= KMAX; ++aa) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m <= aa; ++m)
        if (m <= k) acc += u_of(m, aa) * v[m];
      if (aa <= k) D[aa] = acc;
    }
  };

  // The replay of accepted step m for a cell with act (the others rest);
  // returns the corrected state in y_new (this lane's component) and 0 on a
  // non-finite or singular corrector.  The corrector equation is solved to
  // ADJ_TOL; the iteration keeps the Newton matrix of the predictor while the
  // increments shrink at least kChordRate-fold per iteration and takes a new
  // one (a Newton step) when they do not, so its solution is the exact
  // corrector either way.
  int n_it = 0, n_lu = 0;  // Newton iterations and factorizations of the replay
  auto replay_step = [&](int m, bool act, double &y_new) -> int {
    const int k = act ? so[m] : 1;
    const double hstep = act ? sh[m] : 0.0, ratio = act ? sr[m] : 1.0;
    if (act && ratio != 1.0) rescale_fwd(k, ratio);
    double gk = 1.0;
#pragma unroll
    for (int kk = 1; kk <= KMAX; ++kk)
      if (kk == k) gk = gamma_of(kk);
    double ypred = D[0], sb = 0.0;
#pragma unroll
    for (int j = 1; j <= KMAX; ++j)
      if (j <= k) {
        ypred += D[j];
        sb += gamma_of(j) * D[j];
      }
    const double psi = sb / gk;
    const double isc = 1.0 / (a.atol + a.rtol * fabs(ypred));
    const double c = hstep / gk;
    double d = 0.0, y = ypred, dprev = 0.0;
    int ok = 1, fresh = 1;
    bool done = !act;
    for (int it = 0; it < ADJ_MAXIT; ++it) {
      if (__ballot(!done) == 0) break;  // every cell of the wave is done
      if (!done) ++n_it;
      if (own && !done) ybuf[i] = y;
      double F;
      const int okf = eval_f_m(c, !done, !done && fresh, F);
      if (!done && !okf) {
        ok = 0;
        done = true;
      }
      const bool do_fac = !done && fresh;
      if (do_fac) ++n_lu;
      // (a factorization pass in which no cell of the wave factors changes
      // nothing, so the wave skips it)
      const int nonsing = __ballot(do_fac) != 0 ? factor(do_fac) : 1;
      if (do_fac && !nonsing) {
        ok = 0;
        done = true;
      }
      const double dy = solve(c * F - psi - d);
      const double dn = wrms(dy, isc);
      if (!done) {
        if (!isfinite(dn)) {
          ok = 0;
          done = true;
        } else {
          y += dy;
          d += dy;
          if (dn <= ADJ_TOL) {
            done = true;
          } else {
            fresh = it > 0 && dn > kChordRate * dprev;
            dprev = dn;
          }
        }
      }
    }
    y_new = y;
    // history update (row k+2 of the production integrator only feeds its
    // error estimates, never the solution, so the replay does not keep it)
    if (act) {
#pragma unroll
      for (int kk = 1; kk <= KMAX; ++kk) {
        if (kk == k) {
          D[kk + 1] = d;
#pragma unroll
          for (int j = kk; j >= 0; --j) D[j] += D[j + 1];
        }
      }
    }
    return ok;
  };

  // ---------------- forward replay from y(0) ----------------
  auto init_history = [&]() -> int {
    if (own) ybuf[i] = y0v;
    double f0;
    const int ok = eval_f_m(0.0, true, false, f0);
#pragma unroll
    for (int j = 0; j < DROWS; ++j) D[j] = 0.0;
    D[0] = y0v;
    D[1] = blk[1] * f0;
    return ok;
  };

  if constexpr (!BACKWARD) {
    int ok = init_history();
    const int m_end = wave_max_of_groups<G>(nst);
    double y_new = 0.0;
    for (int m = 0; m < m_end; ++m) {
      const bool act = ok && m < nst;
      if (act && m % CK == 0 && own) {
        double *cp = ck + (size_t)(m / CK) * 7 * n;
#pragma unroll
        for (int j = 0; j < DROWS; ++j) cp[j * n + i] = D[j];
      }
      const int okm = replay_step(m, act, y_new);
      if (act && !okm) ok = 0;
      if (act && has_states && own) yst[(size_t)m * n + i] = y_new;
    }
    if (!dead) {
      if (i == 0 && a.iters) {
        a.iters[cell] = n_it;
        a.iters[C + cell] = n_lu;
      }
      if (!ok) {
        // the outputs keep the recording run's end state; E follows it
        if (i == 0) {
          a.status[cell] = ST_NONFINITE;
          a.Eout[cell] = (a.Tout[cell] - a.T0[cell]) / nt.inv_cv;
        }
      } else if (own) {
        if (i < N) {
          a.Yout[(int64_t)i * C + cell] = D[0];
        } else {
          a.Tout[cell] = D[0];
          a.Eout[cell] = (D[0] - y0v) / nt.inv_cv;
        }
      }
    }
  } else {
    // ---------------- reverse sweep ----------------
    // cotangent of y_end: (gY, c_v gE) on D_0
    double lam[DROWS];
#pragma unroll
    for (int j = 0; j < DROWS; ++j) lam[j] = 0.0;
    if (own && !dead) lam[0] = (i < N) ? a.gY[(int64_t)i * C + cell] : a.gE[cell] / nt.inv_cv;
    for (int r = i; r < R; r += G) grl[r] = 0.0;

    // per reaction: w_r = sum_i W_ir mu_i with mu in vbuf; for cells with
    // act adds scale * R_r * w_r to the gradient and, with want_jt too,
    // scale * w_r * dR_r/dy into jout (J^T mu).  The state is in ybuf.
    auto accumulate = [&](double scale, bool want_jt, bool act) {
      if (want_jt && own) jout[i] = 0.0;
      wave_lds_sync();
      const TPow tp = tpow(ybuf[N]);
      for (int r = i; r < R; r += G) {
        {
          double g[4];
          const double v = rate_and_slots(tb, r, tp, ybuf, rho, want_jt, g);
          const int4 *ro = reinterpret_cast<const int4 *>(tb.rout + 8 * r);
          const int4 r0 = ro[0], r1 = ro[1];
          const int ent[7] = {r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
          double w = tb.qcv[r] * vbuf[N];
          for (int e = 0; e < r0.x; ++e)
            w += (double)(signed char)(ent[e] & 0xff) * vbuf[ent[e] >> 8];
          if (act) grl[r] += scale * v * w;
          if (want_jt) {
            const int *sp = tb.rsp + 4 * r;
            for (int s = 0; s < 4; ++s) {
              const int col = (s < 3) ? sp[s] : N;
              if (col >= 0) lds_add(&jout[col], w * g[s]);
            }
          }
        }
      }
      wave_lds_sync();
    };

    double *segg = a.seg + (size_t)cell * CK * n;  // corrected states of the segment
    const int n_seg = (nst + CK - 1) / CK;
    const int sg_end = wave_max_of_groups<G>(n_seg);
    for (int sg = sg_end - 1; sg >= 0; --sg) {
      const int m0 = sg * CK;
      const int m1 = sg < n_seg ? (m0 + CK < nst ? m0 + CK : nst) : m0;
      // recompute the segment from its checkpoint, keeping y_new (cells
      // whose states the replay kept in the pool skip it)
      if (m1 > m0 && own && !has_states) {
        const double *cp = ck + (size_t)sg * 7 * n;
#pragma unroll
        for (int j = 0; j < DROWS; ++j) D[j] = cp[j * n + i];
      }
      if constexpr (!POOL) {
        for (int mm = 0; mm < CK; ++mm) {
          const bool act = m0 + mm < m1 && !has_states;
          if (__ballot(act) == 0) break;  // later steps of the segment: no cell has them
          double y_new;
          replay_step(m0 + mm, act, y_new);
          if (act && own) segg[mm * n + i] = y_new;
        }
      }
      // walk it backwards
      for (int mm = CK - 1; mm >= 0; --mm) {
        const int m = m0 + mm;
        const bool act = m < m1;
        if (__ballot(act) == 0) continue;
        const double ys = (act && own) ? (has_states ? yst[(size_t)m * n + i] : segg[mm * n + i])
                                       : 1.0;
        const int k = act ? so[m] : 1;
        const double ratio = act ? sr[m] : 1.0;
        double gk = 1.0;
#pragma unroll
        for (int kk = 1; kk <= KMAX; ++kk)
          if (kk == k) gk = gamma_of(kk);
        const double c = act ? sh[m] / gk : 0.0;
        // transpose of the history update D'_{k+1} = d, D'_j = sum_{i=j..k} D_i + d
        double ld = 0.0;
        if (act) {
          double pre[DROWS];
          double run = 0.0;
#pragma unroll
          for (int j = 0; j < DROWS; ++j) {
            run += lam[j];
            pre[j] = run;  // sum_{i<=j} lam_i
          }
#pragma unroll
          for (int kk = 1; kk <= KMAX; ++kk)
            if (kk == k) {
              ld = pre[kk] + lam[kk + 1];
#pragma unroll
              for (int j = 0; j <= kk; ++j) lam[j] = pre[j];
              lam[kk + 1] = 0.0;
            }
        }
        // corrector: mu = M^-T lambda_d at y_new
        if (act && own) ybuf[i] = ys;
        double dummy;
        eval_f_m(c, false, act, dummy);
        factor(act);
        const double mu = solve_t(ld);
        if (own) vbuf[i] = act ? mu : 0.0;
        accumulate(c, act, act);
        if (act) {
          const double ly0 = own ? c * jout[i] : 0.0;
          const double lpsi = -mu;
#pragma unroll
          for (int j = 0; j <= KMAX; ++j)
            if (j <= k) lam[j] += ly0;
#pragma unroll
          for (int j = 1; j <= KMAX; ++j)
            if (j <= k) lam[j] += (gamma_of(j) / gk) * lpsi;
          // transpose of the rescale: lam <- (R(rho) U) lam on rows 0..k
          if (ratio != 1.0) {
            double w[KMAX + 1];
#pragma unroll
            for (int mq = 0; mq <= KMAX; ++mq) {
              double acc = 0.0;
#pragma unroll
              for (int aa = mq; aa <= KMAX; ++aa)
                if (aa <= k) acc += u_of(mq, aa) * lam[aa];
              w[mq] = acc;
            }
            double nl[KMAX + 1];
#pragma unroll
            for (int b = 0; b <= KMAX; ++b) nl[b] = 0.0;
#pragma unroll
            for (int mq = 0; mq <= KMAX; ++mq) {
              if (mq > k) continue;
              const double x = (double)mq * ratio;
              double rb = 1.0;
              nl[0] += w[mq];
#pragma unroll
              for (int b = 1; b <= KMAX; ++b) {
                rb *= ((double)(b - 1) - x) * (1.0 / (double)b);
                if (b <= k) nl[b] += rb * w[mq];
              }
            }
#pragma unroll
            for (int b = 0; b <= KMAX; ++b)
              if (b <= k) lam[b] = nl[b];
          }
        }
      }
    }
    // D_1 = h_init f(y(0)): its multiplier dependence
    if (own) {
      ybuf[i] = y0v;
      vbuf[i] = lam[1];
    }
    accumulate(dead ? 0.0 : blk[1], false, !dead);
    if (!dead)
      for (int r = i; r < R; r += G) a.grad[(int64_t)r * C + cell] = grl[r];
  }
}

__global__ void __launch_bounds__(256) adj_key_kernel(AdjArgs a, float *key) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n_cells) return;
  // fewer accepted steps -> larger key -> later position; 16 steps per
  // octave, i.e. buckets of 8 steps up to ~1,000 steps (longer runs share
  // the first bucket); failed runs (no steps recorded) last
  const double ns = a.sched[c * a.sched_stride];
  key[c] = (ns >= 0.0 && a.status[c] == ST_OK) ? exp2f(-(float)ns * (1.0f / 16.0f))
                                                : __builtin_inff();
}

// Exclusive scan of the cells' state counts (n * recorded steps, 0 for a
// failed recording) in one workgroup: each thread sums a contiguous chunk,
// the workgroup scans the chunk sums in LDS, then each thread writes its
// chunk's offsets (-1 past the pool's capacity).
__global__ void __launch_bounds__(1024) adj_states_kernel(AdjArgs a) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t C = a.n_cells, n = a.net.n;
  const int64_t per = (C + 1023) / 1024;
  const int64_t c0 = t * per < C ? t * per : C, c1 = c0 + per < C ? c0 + per : C;
  auto count = [&](int64_t c) -> int64_t {
    const double ns = a.sched[c * a.sched_stride];
    return (ns > 0.0 && a.status[c] == ST_OK) ? n * (int64_t)ns : 0;
  };
  int64_t sum = 0;
  for (int64_t c = c0; c < c1; ++c) sum += count(c);
  part[t] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan over the 1024 chunk sums
  for (int d = 1; d < 1024; d <<= 1) {
    const int64_t v = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t off = part[t] - sum;
  for (int64_t c = c0; c < c1; ++c) {
    const int64_t k = count(c);
    a.soff[c] = (k > 0 && off + k <= a.states_cap) ? off : -1;
    off += k;
  }
}

__global__ void __launch_bounds__(256) adj_inverse_kernel(const int32_t *pos, int64_t n,
                                                          int32_t *order) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) order[pos[c]] = (int32_t)c;
}

}  // namespace

size_t adjoint_sched_stride(int cap) { return 2 + 2 * (size_t)cap + ((size_t)cap + 1) / 2; }
int adjoint_n_ckpt(int cap) { return (cap + CK - 1) / CK; }
size_t adjoint_seg_doubles(int n) { return (size_t)CK * n; }
size_t adjoint_lds_bytes(int R, int n, int waves) {
  return 8 * (tab_doubles_of(R) + (size_t)waves * adj_wave_doubles(n, R));
}
int adjoint_cells_per_wave(int n) { return 64 / adj_group(n); }

hipError_t launch_record_queue(const BurnArgs &a, int L, int S, int block_waves, int grid,
                               unsigned long long *queue, hipStream_t stream) {
#define BN_RECQ(l, s, w)                                                                         \
  if (L == l && S == s) {                                                                      \
    using SH = Shape<l, s>;                                                                    \
    const size_t lds =                                                                         \
        8 * (tab_doubles_of(a.net.R) + (size_t)block_waves * SH::wave_doubles(a.net.n));       \
    hipLaunchKernelGGL((burn_record_queue_kernel<l, s, w>), dim3((unsigned)grid),              \
                       dim3(64 * block_waves), lds, stream, a, queue);                         \
    return hipGetLastError();                                                                  \
  }
  if (grid < 1) return hipErrorInvalidValue;
  BN_RECQ(8, 1, 2)
  BN_RECQ(16, 1, 2)
  BN_RECQ(32, 1, 2)
  BN_RECQ(64, 1, 1)
#undef BN_RECQ
  return hipErrorInvalidValue;
}

hipError_t launch_adjoint_order(const AdjArgs &a, float *key, int32_t *pos, unsigned *hist,
                                int32_t *order, hipStream_t stream) {
  const int64_t n = a.n_cells;
  if (n <= 0) return hipSuccess;
  if (n > 0x7fffffff) return hipErrorInvalidValue;
  hipError_t e = launch_zero(reinterpret_cast<unsigned long long *>(hist), ORDER_BUCKETS, stream);
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(adj_key_kernel, dim3(blocks), dim3(256), 0, stream, a, key);
  e = launch_sort_keys(key, n, pos, hist, stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adj_inverse_kernel, dim3(blocks), dim3(256), 0, stream, pos, n, order);
  return hipGetLastError();
}

hipError_t launch_adjoint_states(const AdjArgs &a, hipStream_t stream) {
  if (a.n_cells <= 0) return hipSuccess;
  hipLaunchKernelGGL(adj_states_kernel, dim3(1), dim3(1024), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_adjoint(const AdjArgs &a0, bool backward, int waves, int simd_waves,
                          hipStream_t stream) {
  const size_t lds = adjoint_lds_bytes(a0.net.R, a0.net.n, waves);
  const int G = adj_group(a0.net.n);
  const int64_t per_block = (int64_t)waves * (64 / G);
  const int64_t blocks = (a0.n_cells + per_block - 1) / per_block;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks), block(64 * waves);
  const bool w3 = simd_waves >= 3;
  AdjArgs a = a0;
#define BN_ADJ(bwd, w, g, pool) \
  hipLaunchKernelGGL((adjoint_kernel<bwd, w, g, pool>), grid, block, lds, stream, a)
  if (!backward) {
    a.part = 0;
    if (G == 32) {
      if (w3) BN_ADJ(false, 3, 32, false);
      else BN_ADJ(false, 2, 32, false);
    } else {
      if (w3) BN_ADJ(false, 3, 64, false);
      else BN_ADJ(false, 2, 64, false);
    }
    return hipGetLastError();
  }
  // Reverse sweep: with a pool, the cells whose states it holds run in the
  // instance without the segment recomputation (fewer registers, no spills
  // at three waves per SIMD), then the others in the full instance.
  const bool split = a0.states != nullptr && a0.soff != nullptr && a0.states_cap > 0;
  if (split) {
    a.part = 1;
    if (G == 32) {
      if (w3) BN_ADJ(true, 3, 32, true);
      else BN_ADJ(true, 2, 32, true);
    } else {
      if (w3) BN_ADJ(true, 3, 64, true);
      else BN_ADJ(true, 2, 64, true);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  a.part = split ? 2 : 0;
  if (G == 32) {
    if (w3) BN_ADJ(true, 3, 32, false);
    else BN_ADJ(true, 2, 32, false);
  } else {
    if (w3) BN_ADJ(true, 3, 64, false);
    else BN_ADJ(true, 2, 64, false);
  }
#undef BN_ADJ
  return hipGetLastError();
}

}  // namespace bn
