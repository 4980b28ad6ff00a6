// burn_gen_body.h -- device code of the burn for one network whose rates,
// right-hand side and Jacobian are generated as straight-line code with the
// stoichiometry, rate coefficients and sparsity known at compile time (the
// per-network code generation of Sec. 2 of the paper).  The library writes a
// source per network (struct GenNet, see below), appends it to this body and
// compiles it for gfx950 at run time.
//
// The integrator is the one of the table-driven kernels, decision by
// decision: variable-order (1..5) BDF in backward differences, modified
// Newton, partially pivoted LU of I - cJ, the same controller and counters.
//
// Mapping onto a 64-wide wavefront.  A cell is owned by LPC lanes (1 or 2):
// component i lives on lane i % LPC, slot i / LPC (NS = ceil(n / LPC) slots
// per lane).  The lanes of a cell split the rate exponentials (lane h takes
// reactions t LPC + h, its coefficients read from an LDS table) and
// broadcast them; the rest of the generated code is the same in every lane
// (so the wave stays converged), and each lane keeps its own components of
// the right-hand side and its own rows of the Newton matrix.
// Per lane:
//   * registers: the entries of its LU rows that the fill pattern allows
//     (the others are zero constants), their reciprocal pivots, and the
//     Newton iterate and correction of its components;
//   * LDS: the backward-difference history, then psi and the reciprocal
//     error scales, laid out [row][slot][lane] so a wave's access to one
//     (row, slot) is 64 consecutive doubles whatever row each cell reads (no
//     bank conflicts);
//   * global memory: its Jacobian rows (written when J is evaluated, read
//     when I - cJ is formed for a new step size), and a scratch area for the
//     rare factorization that pivots off the diagonal.
// The factorization runs with the pivots on the diagonal, the fill pattern of
// that ordering known at compile time.  Partial pivoting (the first largest
// magnitude, so the diagonal wins ties) chooses the diagonal at column K
// exactly when no entry below it is larger in magnitude, i.e. when every
// multiplier l_iK = a_iK / a_KK has |l_iK| <= 1; the multipliers are formed
// anyway (as a_iK times the reciprocal pivot, within two units in the last
// place of the quotient), and one of magnitude >= 1 - 2^-51 (or NaN) marks
// the cell.  That flags every factorization whose pivots leave the diagonal
// and, rarely, one with a near-tie.  A marked cell factors I - cJ again from
// the start with row interchanges in its scratch area, where the factors
// stay (dense, rows permuted) and its solves read them.  Either way the
// pivots are the ones partial pivoting chooses.
#pragma once

#include "bn_math.h"
#include "burn_gen_args.h"

namespace bng {

constexpr double kSafety = 0.9;
constexpr double kMinFactor = 0.2;
constexpr double kMaxFactor = 10.0;
constexpr double kNewtonTol = 0.03;
constexpr int kNewtonMaxIt = 4;
constexpr int KMAX = 5;
constexpr int DROWS = KMAX + 2;  // D_0 .. D_{k+1}; D_{k+2} is formed and used at once
// LDS rows per slot: the history, psi, the reciprocal error scales, then
// (when the LDS holds them, see VecLds) the Newton correction and the
// reciprocal pivots
constexpr int ROW_PSI = DROWS, ROW_ISC = DROWS + 1, ROW_DD = DROWS + 2, ROW_DINV = DROWS + 3;
constexpr int LDS_BYTES = 160 * 1024;

// Doubles at the head of the LDS: the rate multipliers (R rounded up to 8),
// then, when the LPC lanes of a cell split the rate exponentials, the rate
// coefficient table (8 per reaction, reactions padded to a multiple of LPC),
// then the reciprocals 1/j of j = 0..7 (RECIP doubles; entry 0 unused).
constexpr int RECIP = 8;
constexpr int head_doubles(int R, int LPC) {
  return (R + 7) / 8 * 8 + (LPC > 1 ? (R + LPC - 1) / LPC * LPC * 8 : 0) + RECIP;
}
// rows per slot in LDS for a system with NS slots and R reactions: the
// Newton correction and the reciprocal pivots go there too when four waves
// of it fit (it frees registers for the right-hand side)
constexpr int lds_rows(int NS, int R, int LPC) {
  return (8 * (head_doubles(R, LPC) + 4 * (DROWS + 4) * NS * 64) <= LDS_BYTES) ? DROWS + 4
                                                                                : DROWS + 2;
}
constexpr long long lds_bytes(int NS, int R, int LPC) {
  return 8LL * (head_doubles(R, LPC) + 4LL * lds_rows(NS, R, LPC) * NS * 64);
}
constexpr int XCD_PARTS = 8;

enum { PH_F0 = 0, PH_F1 = 1, PH_NEWTON = 2, PH_DONE = 3, PH_LOAD = 4, PH_IDLE = 5 };
enum { ST_OK = 0, ST_MAX_STEPS = 1, ST_UNDERFLOW = 2, ST_NONFINITE = 3, ST_BAD_INPUT = 4 };
enum { CNT_STEPS = 0, CNT_REJ, CNT_NFAIL, CNT_RHS, CNT_JAC, CNT_LU, CNT_SOLVE, CNT_ORDER };

// gamma_k = sum_{j=1..k} 1/j, summed in ascending j.
constexpr double gamma_of(int k) {
  double g = 0.0;
  for (int j = 1; j <= k; ++j) g += 1.0 / (double)j;
  return g;
}

// U = R(1) of the step-change transform: U[i][j] = prod_{m=1..i} (m-1-j)/m.
constexpr double u_of(int i, int j) {
  double v = 1.0;
  for (int m = 1; m <= i; ++m) v *= (double)(m - 1 - j) / (double)m;
  return v;
}

// 1 / d from the hardware estimate and two Newton steps (within about one
// unit in the last place; used where the quotient only scales a norm or
// forms an LU multiplier, never where the integrator's definition fixes a
// correctly rounded result).  d = 0 gives NaN, as does d = inf.
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// x / d for a small positive integer d with r = 1 / d rounded: the product,
// then one remainder step (the remainder is exact and the corrected
// quotient is the rounded x / d whenever that is a normal number).
__device__ __forceinline__ double divq(double x, double d, double r) {
  const double q = x * r;
  const double rem = fma(-q, d, x);
  return fma(rem, r, q);
}

template <int N>
struct Unroll {
  template <class F>
  __device__ __forceinline__ static void run(F &&f) {
    Unroll<N - 1>::run(f);
    f.template operator()<N - 1>();
  }
};
template <>
struct Unroll<0> {
  template <class F>
  __device__ __forceinline__ static void run(F &&) {}
};

// DPP quad permutes (bound_ctrl: a lane reading an inactive lane gets 0; the
// two lanes of a pair are always active together).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
// a pointer into device global memory (address space 1), so the accesses
// through it are global (not flat) instructions
typedef __attribute__((address_space(1))) double *gptr;
typedef const __attribute__((address_space(1))) double *gcptr;
typedef __attribute__((address_space(1))) int *giptr;

constexpr int QP_XOR1 = 0xB1;  // [1,0,3,2]
constexpr int QP_EVEN = 0xA0;  // [0,0,2,2]
constexpr int QP_ODD = 0xF5;   // [1,1,3,3]

// Operations over the LPC lanes of a cell.
template <int LPC>
struct Grp;
template <>
struct Grp<1> {
  __device__ __forceinline__ static double sum(double v) { return v; }
  __device__ __forceinline__ static double max_nonnan(double v) { return v; }
  __device__ __forceinline__ static int any(int v) { return v; }
  template <int SRC>
  __device__ __forceinline__ static double bcast(double v) {
    return v;
  }
};
template <>
struct Grp<2> {
  // a + b in one lane, b + a in the other: the same double
  __device__ __forceinline__ static double sum(double v) { return v + dpp_f64<QP_XOR1>(v); }
  // the larger of the two (values are >= -1 and never NaN)
  __device__ __forceinline__ static double max_nonnan(double v) {
    const double o = dpp_f64<QP_XOR1>(v);
    return o > v ? o : v;
  }
  __device__ __forceinline__ static int any(int v) { return v | dpp_i32<QP_XOR1>(v); }
  template <int SRC>
  __device__ __forceinline__ static double bcast(double v) {
    return dpp_f64<SRC ? QP_ODD : QP_EVEN>(v);
  }
};

// One wave burns its cells.  NET is the generated network:
//   N, R, n = N + 1                 sizes
//   ufill[NS]                       per slot, the union over its rows of the
//                                   LU fill pattern with diagonal pivots
//                                   (bit j: column j may be nonzero)
//   fpat[n]                         that pattern row by row
//   rhs(y, rho, em, h, F)           F = own components of f(y)
//   jac_m(y, rho, em, h, cc, M, jb, stride, jbad)
//                                   J(y): own rows into the workspace
//                                   (entry E at jb[E * stride]), and
//                                   M = I - cc J into M; jbad = any J entry
//                                   of the own rows not finite
//   load_m(h, cc, M, jb, stride)
//                                   M = I - cc J from the workspace
// em[R] are the rate multipliers exp(p_r) (ones without multipliers).
template <class NET, int LPC>
__device__ __forceinline__ void run_cells(const GenArgs &a, const double *em, double *Dw) {
  constexpr int n = NET::n, N = NET::N;
  constexpr int NS = (n + LPC - 1) / LPC;
  using G = Grp<LPC>;
  // the reciprocals 1/j at the end of the LDS head (the order-dependent
  // quotients of the controller read them instead of dividing)
  const double *recip = em + head_doubles(NET::R, LPC) - RECIP;

  const int lane = threadIdx.x & 63;
  int h = LPC == 2 ? (lane & 1) : 0;  // made opaque in every iteration (see below)
  const int cw = lane / LPC;           // cell slot of the wave
  const long long at = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // workspace column

  // launch constants, each kept in scalar registers of its own
  long long C = a.n_cells;
  double rtol = a.rtol, atol = a.atol, t_end = a.t_end;
  // (global, not flat, pointers: a flat access also counts as an LDS
  // access, so an LDS wait after a flat store would wait for the store)
  gptr gY = (gptr)a.Y, gT = (gptr)a.T;
  gcptr grho = (gcptr)a.rho;
  giptr gst = (giptr)a.status, gcnt = (giptr)a.counters;
  int max_steps = a.max_steps;
  asm volatile("" : "+s"(C), "+s"(rtol), "+s"(atol), "+s"(t_end));
  asm volatile("" : "+s"(gY), "+s"(gT), "+s"(grho), "+s"(gst), "+s"(gcnt), "+s"(max_steps));
  const long long NL = a.n_lanes;
  // this lane's column of the workspaces
  const gptr jws = (gptr)(a.jws + at), lws = (gptr)(a.lws + at);
  // A workspace address is loop-invariant, so the compiler would compute
  // every entry's address once before the cell loop and keep them all in
  // registers; the blocks that touch a workspace take their base pointer
  // through an empty asm instead, which keeps the addresses inside them.
  auto opaque = [](gptr p) __attribute__((always_inline)) {
    asm volatile("" : "+v"(p));
    return p;
  };
  // the lane stride likewise (else every entry's offset is a scalar kept
  // across the loop)
  auto stride = [&]() __attribute__((always_inline)) {
    long long v = NL;
    asm volatile("" : "+s"(v));
    return v;
  };

  auto comp = [&](int s) __attribute__((always_inline)) { return s * LPC + h; };
  // comp(s) > K, comp(s) < K and comp(s) < n with the slot s and K known at
  // compile time: the slot decides unless K lies in it (h is opaque to the
  // compiler, so comp(s) itself is never folded)
  auto above = [&](int s, int K) __attribute__((always_inline)) {
    return s > K / LPC ? true : (s < K / LPC ? false : h > K % LPC);
  };
  auto below = [&](int s, int K) __attribute__((always_inline)) {
    return s < K / LPC ? true : (s > K / LPC ? false : h < K % LPC);
  };
  auto real = [&](int s) __attribute__((always_inline)) {
    return s * LPC + LPC - 1 < n ? true : (s * LPC >= n ? false : h < n - s * LPC);
  };
  auto Dref = [&](int row, int s) __attribute__((always_inline)) -> double & {
    return Dw[(row * NS + s) * 64 + lane];
  };

  // ---- per-lane state
  constexpr bool VEC_LDS = lds_rows(NS, NET::R, LPC) == DROWS + 4;
  double LU[NS][n];  // rows comp(s) of the factors (diagonal pivots)
  double dinv_r[VEC_LDS ? 1 : NS], dd_r[VEC_LDS ? 1 : NS];  // when not in LDS
  double yv[NS], F[NS];
  // the reciprocal pivots of the LU rows and the Newton correction
  auto dinv = [&](int s) __attribute__((always_inline)) -> double & {
    if constexpr (VEC_LDS) return Dref(ROW_DINV, s);
    else return dinv_r[s];
  };
  auto dd = [&](int s) __attribute__((always_inline)) -> double & {
    if constexpr (VEC_LDS) return Dref(ROW_DD, s);
    else return dd_r[s];
  };
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    dinv(s) = 1.0;
#pragma unroll
    for (int j = 0; j < n; ++j) LU[s][j] = 0.0;
    dd(s) = yv[s] = F[s] = 0.0;
  }
  int cnt[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) cnt[c] = 0;
  int perm = 0;   // the factors are the pivoting path's, in the scratch area
  int jr_ok = 0;  // the workspace holds J(y_J) of this cell
  int yj_pred = 0;  // y_J is the predictor (else D_0)
  int k = 1;

  // the predictor sum_{j <= k} D_j of slot s, in ascending j
  auto pred = [&](int s) __attribute__((always_inline)) {
    double sa = Dref(0, s);
    double dr[KMAX + 1];
#pragma unroll
    for (int j = 1; j <= KMAX; ++j) dr[j] = Dref(j, s);
#pragma unroll
    for (int j = 1; j <= KMAX; ++j)
      if (j <= k) sa += dr[j];
    return sa;
  };

  // full vector from the own components of every lane of the cell
  auto gather = [&](const double(&v)[NS], double(&y)[n]) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (s * LPC < n) y[s * LPC] = G::template bcast<0>(v[s]);
      if constexpr (LPC == 2) {
        if (s * LPC + 1 < n) y[s * LPC + 1] = G::template bcast<1>(v[s]);
      }
    }
  };

  // weighted mean square over the n components (inv = 1 / scale), and its
  // square root, the weighted RMS norm
  auto wms = [&](const double(&v)[NS], const double(&inv)[NS]) __attribute__((always_inline)) {
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double z = v[s] * inv[s];
      if (real(s)) acc += z * z;
    }
    return divq(G::sum(acc), (double)n, 1.0 / (double)n);
  };
  auto wrms = [&](const double(&v)[NS], const double(&inv)[NS]) __attribute__((always_inline)) {
    return sqrt(wms(v, inv));
  };

  // change of step size by ratio rh on rows 0..k of D: D <- (R(rh) U)^T D.
  // The (k+1) x (k+1) matrix is the same for every component, so it is
  // formed once: R(rh)[m][b] = prod_{j=1..b} (j - 1 - m rh) / j (row 0 is
  // e_0), U[m][a] = u_of(m, a), and D'_a = sum_b (sum_{m<=a} U[m][a]
  // R[m][b]) D_b for a <= k (rows b > k are zero).
  auto rescale = [&](int k, double rh) __attribute__((always_inline)) {
    double rb[KMAX + 1][KMAX + 1];
#pragma unroll
    for (int m = 1; m <= KMAX; ++m) {
      const double x = (double)m * rh;
      double v = 1.0;
#pragma unroll
      for (int b = 1; b <= KMAX; ++b) {
        v *= ((double)(b - 1) - x) * (1.0 / (double)b);
        rb[m][b] = v;
      }
    }
    double ru[KMAX + 1][KMAX + 1];  // ru[a][b]
#pragma unroll
    for (int aa = 0; aa <= KMAX; ++aa) {
      ru[aa][0] = u_of(0, aa);
#pragma unroll
      for (int m = 1; m <= aa; ++m) ru[aa][0] += u_of(m, aa);
#pragma unroll
      for (int b = 1; b <= KMAX; ++b) {
        double acc = 0.0;
#pragma unroll
        for (int m = 1; m <= aa; ++m) acc += u_of(m, aa) * rb[m][b];
        ru[aa][b] = acc;
      }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double dcol[KMAX + 1];
#pragma unroll
      for (int b = 0; b <= KMAX; ++b) {
        const double x = Dref(b, s);
        dcol[b] = (b <= k) ? x : 0.0;
      }
#pragma unroll
      for (int aa = 0; aa <= KMAX; ++aa) {
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b <= KMAX; ++b) acc += ru[aa][b] * dcol[b];
        if (aa <= k) Dref(aa, s) = acc;
      }
    }
  };

  double rho = 1.0;

  // ---- right-hand side F = f(yv) (own components); 1 if finite
  auto rhs = [&]() __attribute__((always_inline)) -> int {
    double y[n];
    gather(yv, y);
    NET::rhs(y, rho, em, h, F);
    int bad = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (real(s) && !__builtin_isfinite(F[s])) bad = 1;
    return !G::any(bad);
  };

  // The pivoting path's scratch area of this lane (base pointer lb): [n][n]
  // factors in position order, n reciprocal pivots, the natural row of every
  // position, then a right-hand side and a solution (n doubles each).
  long long ls = NL;  // the scratch blocks' stride (set opaquely in each)
  auto W = [&](gptr lb, int i, int j) __attribute__((always_inline)) -> __attribute__((address_space(1))) double & {
    return lb[((long long)i * n + j) * ls];
  };
  auto Wd = [&](gptr lb, int i) __attribute__((always_inline)) -> __attribute__((address_space(1))) double & {
    return lb[((long long)n * n + i) * ls];
  };
  auto Wp = [&](gptr lb, int i) __attribute__((always_inline)) -> __attribute__((address_space(1))) double & {
    return lb[((long long)n * n + n + i) * ls];
  };
  auto Wt = [&](gptr lb, int i) __attribute__((always_inline)) -> __attribute__((address_space(1))) double & {
    return lb[((long long)n * n + 2 * n + i) * ls];
  };
  auto Wx = [&](gptr lb, int i) __attribute__((always_inline)) -> __attribute__((address_space(1))) double & {
    return lb[((long long)n * n + 3 * n + i) * ls];
  };

  // ---- M x = b with the factors (b natural order in, x natural order out):
  // register factors with the compile-time fill pattern (diagonal pivots)
  auto solve_reg = [&](double(&b)[NS]) __attribute__((always_inline)) {
    // forward substitution with the unit lower factor
    Unroll<n>::run([&]<int K>() __attribute__((always_inline)) {
      constexpr int ks = K / LPC, kh = K % LPC;
      bool used = false;
#pragma unroll
      for (int s = ks; s < NS; ++s) used = used || ((NET::ufill[s] >> K) & 1ull);
      if (used) {
        const double xk = G::template bcast<kh>(b[ks]);
#pragma unroll
        for (int s = ks; s < NS; ++s) {
          if ((NET::ufill[s] >> K) & 1ull) {
            const double lk = above(s, K) ? LU[s][K] : 0.0;
            b[s] = fma(-lk, xk, b[s]);
          }
        }
      }
    });
    // back substitution with the upper factor: x_K = b_K / U_KK goes to the
    // components above it; each lane scales its own components at the end
    // (the same product)
    Unroll<n>::run([&]<int KK>() __attribute__((always_inline)) {
      constexpr int K = n - 1 - KK;
      constexpr int ks = K / LPC, kh = K % LPC;
      bool used = false;
#pragma unroll
      for (int s = 0; s <= ks; ++s) used = used || ((NET::ufill[s] >> K) & 1ull);
      if (used) {
        const double xk = G::template bcast<kh>(b[ks] * dinv(ks));
#pragma unroll
        for (int s = 0; s <= ks; ++s) {
          if ((NET::ufill[s] >> K) & 1ull) {
            const double uk = below(s, K) ? LU[s][K] : 0.0;
            b[s] = fma(-uk, xk, b[s]);
          }
        }
      }
    });
#pragma unroll
    for (int s = 0; s < NS; ++s) b[s] = b[s] * dinv(s);
  };
  // the same with the pivoting path's factors: the whole system in every
  // lane of the cell, the same operations row by row, in the scratch area
  // (a rare path: plain loops, nothing held in registers)
  auto solve_mem = [&](double(&b)[NS]) __attribute__((always_inline)) {
    const gptr lb = opaque(lws);
    ls = stride();
    {
      double x[n];
      gather(b, x);
#pragma unroll
      for (int i = 0; i < n; ++i) Wt(lb, i) = x[i];
    }
#pragma unroll 1
    for (int i = 0; i < n; ++i) {
      double v = Wt(lb, (int)Wp(lb, i));
#pragma unroll 1
      for (int j = 0; j < i; ++j) v = fma(-W(lb, i, j), Wx(lb, j), v);
      Wx(lb, i) = v;
    }
#pragma unroll 1
    for (int i = n - 1; i >= 0; --i) {
      double v = Wx(lb, i);
#pragma unroll 1
      for (int j = n - 1; j > i; --j) v = fma(-W(lb, i, j), Wx(lb, j), v);
      Wx(lb, i) = v * Wd(lb, i);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) b[s] = comp(s) < n ? Wx(lb, comp(s)) : 0.0;
  };
  auto solve = [&](double(&b)[NS]) __attribute__((always_inline)) {
    if (__ballot(perm) == 0) {
      solve_reg(b);
    } else if (perm) {
      solve_mem(b);
    } else {
      solve_reg(b);
    }
  };

  // ---- the factorization of M (in LU) for the cells that want one, with
  // diagonal pivots and the compile-time fill pattern; dev = 1 where a
  // multiplier shows that partial pivoting would leave the diagonal (or
  // nearly ties it)
  auto factor_diag = [&](int &dev, int &fsing) __attribute__((always_inline)) {
    constexpr double kTie = 1.0 - 0x1p-51;
#pragma unroll
    for (int s = 0; s < NS; ++s) dinv(s) = 1.0;
    Unroll<n>::run([&]<int K>() __attribute__((always_inline)) {
      constexpr int ks = K / LPC, kh = K % LPC;
      constexpr unsigned long long prow = NET::fpat[K];
      const double dg = G::template bcast<kh>(LU[ks][K]);
      if (!(fabs(dg) > 0.0)) fsing = 1;
      const double rinv = rcp_nr(dg);
      if (!above(ks, K) && !below(ks, K)) dinv(ks) = rinv;
      double P[n];
#pragma unroll
      for (int j = K + 1; j < n; ++j)
        if ((prow >> j) & 1ull) P[j] = G::template bcast<kh>(LU[ks][j]);
#pragma unroll
      for (int s = ks; s < NS; ++s) {
        if ((NET::ufill[s] >> K) & 1ull) {
          if (above(s, K)) {
            const double l = LU[s][K] * rinv;
            if (!(fabs(l) < kTie)) dev = 1;
            LU[s][K] = l;
#pragma unroll
            for (int j = K + 1; j < n; ++j)
              if ((prow >> j) & 1ull) LU[s][j] = fma(-l, P[j], LU[s][j]);
          }
        }
      }
    });
    dev = G::any(dev);
  };

  // Factor M (in LU) with row interchanges (partial pivoting: the first
  // largest |entry| in position order) in this lane's scratch area, where
  // the factors stay.  Both lanes of a cell do the same work on their own
  // copies.
  auto factor_pivot = [&](int &fsing) __attribute__((always_inline)) {
    const gptr lb = opaque(lws);
    ls = stride();
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
      for (int j = 0; j < n; ++j) {
        const double v = LU[s][j];
        const double v0 = G::template bcast<0>(v);
        if (s * LPC < n) W(lb, s * LPC, j) = v0;
        if constexpr (LPC == 2) {
          const double v1 = G::template bcast<1>(v);
          if (s * LPC + 1 < n) W(lb, s * LPC + 1, j) = v1;
        }
      }
    }
#pragma unroll 1
    for (int i = 0; i < n; ++i) Wp(lb, i) = (double)i;
#pragma unroll 1
    for (int K = 0; K < n; ++K) {
      int p = K;
      double best = fabs(W(lb, K, K));
#pragma unroll 1
      for (int i = K + 1; i < n; ++i) {
        const double v = fabs(W(lb, i, K));
        if (v > best) {
          best = v;
          p = i;
        }
      }
      if (!(best > 0.0)) {
        fsing = 1;
        break;
      }
      if (p != K) {
#pragma unroll 1
        for (int j = 0; j < n; ++j) {
          const double t0 = W(lb, K, j);
          W(lb, K, j) = W(lb, p, j);
          W(lb, p, j) = t0;
        }
        const double t1 = Wp(lb, K);
        Wp(lb, K) = Wp(lb, p);
        Wp(lb, p) = t1;
      }
      const double rinv = 1.0 / W(lb, K, K);
      Wd(lb, K) = rinv;
#pragma unroll 1
      for (int i = K + 1; i < n; ++i) {
        const double l = W(lb, i, K) * rinv;
        W(lb, i, K) = l;
#pragma unroll 1
        for (int j = K + 1; j < n; ++j) W(lb, i, j) = fma(-l, W(lb, K, j), W(lb, i, j));
      }
    }
  };

  // ================= cell state machine =================
  long long cell = -1;
  int spent = 0;  // XCD parts of the queue this lane found exhausted (bit x)
  int phase = PH_LOAD;
  int status = 0, write_state = 0;
  int n_eq = 0, jac_cur = 0, lu_ok = 0, it = 0, need_attempt = 0, new_step = 0;
  int fresh_newton = 0, first_jac = 0;
  int have_f = 0;     // F holds the waiting cell's first Newton RHS (1 finite, 2 not)
  int lu_waited = 0;  // iterations this cell has waited for its factorization
  double t = 0.0, hs = 0.0, t_new = 0.0, cc = 0.0, dprev = 0.0, h0 = 0.0, d1 = 0.0;

  auto write_out = [&]() __attribute__((always_inline)) {
    // the rows' offsets from an opaque count, so they are formed here and not
    // kept from before the cell loop
    long long C = a.n_cells;
    asm volatile("" : "+s"(C));
    if (write_state) {
      cnt[CNT_ORDER] = k;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int i = comp(s);
        if (i < N) gY[(long long)i * C + cell] = Dref(0, s);
        else if (i == N) gT[cell] = Dref(0, s);
      }
    }
    if (h == 0) {
      if (gst) gst[cell] = status;
      if (gcnt) {
#pragma unroll
        for (int c = 0; c < 8; ++c)
          gcnt[(long long)c * C + cell] = (status == ST_BAD_INPUT) ? 0 : cnt[c];
      }
    }
  };

  auto load_cell = [&](long long c) __attribute__((always_inline)) {
    if (c >= C) {
      phase = PH_IDLE;
      return;
    }
    long long C = a.n_cells;
    asm volatile("" : "+s"(C));
    cell = c;
    rho = grho[cell];
    status = 0;
    write_state = 0;
    k = 1;
    n_eq = jac_cur = lu_ok = it = need_attempt = new_step = fresh_newton = first_jac = 0;
    have_f = lu_waited = 0;
    jr_ok = yj_pred = 0;
    t = hs = t_new = cc = dprev = h0 = d1 = 0.0;
#pragma unroll
    for (int c8 = 0; c8 < 8; ++c8) cnt[c8] = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = comp(s);
      yv[s] = (i < N) ? gY[(long long)i * C + cell] : ((i == N) ? gT[cell] : 0.0);
    }
    int bad = !(rho > 0.0) || !__builtin_isfinite(rho);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = comp(s);
      if (i < n && !__builtin_isfinite(yv[s])) bad = 1;
      if (i == N && !(yv[s] > 0.0)) bad = 1;
    }
    if (G::any(bad)) {
      status = ST_BAD_INPUT;
      phase = PH_DONE;
    } else {
      phase = PH_F0;
    }
  };

  while (true) {
    // The lane's half index is made opaque once per iteration, so the lane
    // predicates of the unrolled loops are formed where they are used
    // instead of being hoisted out of the loop as scalar masks.
    asm volatile("" : "+v"(h));
    // ---------------- 0: write a finished cell, take the next one ----------------
    if (phase == PH_DONE) {
      write_out();
      phase = PH_LOAD;
    }
    {
      const unsigned long long lmask = __ballot(phase == PH_LOAD && h == 0);
      if (lmask && a.parts) {
        // ordered launch: this workgroup's XCD part first, then the others
        if (phase == PH_LOAD) {
          long long got = -1;
          if (h == 0) {
            const int x0 = (int)(blockIdx.x % XCD_PARTS);
            const long long per = C / XCD_PARTS, extra = C % XCD_PARTS;
            for (int tt = 0; tt < XCD_PARTS && got < 0; ++tt) {
              const int x = (x0 + tt) % XCD_PARTS;
              if ((spent >> x) & 1) continue;  // a part seen exhausted stays so
              const long long count = per + (x < extra ? 1 : 0);
              const unsigned long long i = atomicAdd(&a.parts[x], 1ULL);
              if ((long long)i < count) got = x * per + (x < extra ? x : extra) + (long long)i;
              else spent |= 1 << x;
            }
          }
          got = __builtin_bit_cast(long long, G::template bcast<0>(__builtin_bit_cast(double, got)));
          load_cell(got >= 0 && got < C ? got : C);
        }
      } else if (lmask) {
        // one atomic per wave; the requesting cells take consecutive indices
        const int leader = __ffsll((long long)lmask) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(a.queue, (unsigned long long)__popcll(lmask));
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(base & 0xffffffffULL), leader);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(base >> 32), leader);
        base = ((unsigned long long)hi << 32) | lo;
        const unsigned long long below = lmask & ((1ULL << (cw * LPC)) - 1ULL);
        const unsigned long long idx = base + (unsigned long long)__popcll(below);
        if (phase == PH_LOAD) load_cell(idx < (unsigned long long)C ? (long long)idx : C);
      }
    }
    if (__ballot(phase != PH_IDLE) == 0) break;

    // ---------------- A: start of a step attempt ----------------
    if (phase == PH_NEWTON && need_attempt) {
      if (new_step && cnt[CNT_STEPS] >= max_steps) {
        status = ST_MAX_STEPS;
        phase = PH_DONE;
      } else {
        // step underflow (also catches a non-finite step): 10 ulp(t), t >= 0
        const double ulp = __builtin_bit_cast(double, __builtin_bit_cast(long long, t) + 1LL) - t;
        if (!(hs >= 10.0 * ulp)) {
          status = ST_UNDERFLOW;
          phase = PH_DONE;
        } else {
          t_new = t + hs;
          if (t_new > t_end) {
            t_new = t_end;
            rescale(k, (t_end - t) / hs);
            hs = t_end - t;
            n_eq = 0;
            lu_ok = 0;
          }
          double gk = 1.0, igk = 1.0;
#pragma unroll
          for (int kk = 1; kk <= KMAX; ++kk)
            if (kk == k) {
              gk = gamma_of(kk);
              igk = 1.0 / gamma_of(kk);
            }
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const double sa = pred(s);
            double sb = 0.0;
#pragma unroll
            for (int j = 1; j <= KMAX; ++j)
              if (j <= k) sb += gamma_of(j) * Dref(j, s);
            Dref(ROW_PSI, s) = sb * igk;
            Dref(ROW_ISC, s) = rcp_nr(atol + rtol * fabs(sa));
            dd(s) = 0.0;
            yv[s] = sa;
          }
          cc = hs / gk;
          it = 0;
          need_attempt = 0;
          new_step = 0;
          fresh_newton = 1;
        }
      }
    }

    // ---------------- B: factorizations ----------------
    // A pass costs the wave about the same for one cell as for all of them,
    // so a cell that wants a factorization may wait while the other cells
    // step on: the pass runs once lu_batch cells want one, once a cell has
    // waited lu_wait iterations, or when no other cell has work.  A waiting
    // cell meanwhile evaluates its first Newton RHS (at the predictor, which
    // the wait leaves unchanged); its own arithmetic is the same whether it
    // waits or not.
    const int want = (phase == PH_NEWTON && fresh_newton && !lu_ok);
    int run = 0;
    {
      const unsigned long long wmask = __ballot(want);
      if (wmask != 0) {
        const int others =
            __ballot((phase == PH_F0 || phase == PH_F1 || phase == PH_NEWTON) && !want) != 0;
        run = !others || __popcll(wmask) >= (unsigned)(a.lu_batch * LPC) ||
              __ballot(want && lu_waited >= a.lu_wait) != 0;
      }
    }
    const int fac = want && run;
    int sing = 0;
    if (run) {
      int jbad = 0;
      const int asmj = fac && !jr_ok;
      if (__ballot(asmj) != 0) {
        if (asmj) {
          // J(y_J) for the cells whose Jacobian was refreshed: into the
          // workspace, and I - cJ into the LU registers
          double yo[NS], y[n];
#pragma unroll
          for (int s = 0; s < NS; ++s) yo[s] = yj_pred ? pred(s) : Dref(0, s);
          gather(yo, y);
          NET::jac_m(y, rho, em, h, cc, LU, opaque(jws), stride(), jbad);
          jbad = G::any(jbad);
          jr_ok = 1;
        }
      }
      if (__ballot(fac && !asmj) != 0) {
        if (fac && !asmj) NET::load_m(h, cc, LU, opaque(jws), stride());
      }
      int dev = 0;
      if (fac) {
        factor_diag(dev, sing);
        perm = 0;
      }
      if (__ballot(dev) != 0) {
        if (dev) {
          // again from I - cJ, with row interchanges
          NET::load_m(h, cc, LU, opaque(jws), stride());
          sing = 0;
          factor_pivot(sing);
          perm = 1;
        }
      }
      if (fac) {
        lu_waited = 0;
        if (first_jac && jbad) {
          // the Jacobian at the initial state is not finite
          status = ST_NONFINITE;
          phase = PH_DONE;
          write_state = 0;
        } else {
          cnt[CNT_LU]++;
          lu_ok = 1;
        }
        first_jac = 0;
      }
    }

    double pend = 0.0;
    // a singular Newton matrix is a failed Newton attempt (no RHS needed)
    int nfail = (fac && phase == PH_NEWTON && sing) ? 1 : 0;
    // a waiting cell's RHS that its factorization made moot (a singular
    // matrix, or a non-finite Jacobian at the initial state) was never part
    // of the integration
    if (fac && have_f && (nfail || phase != PH_NEWTON)) {
      cnt[CNT_RHS]--;
      have_f = 0;
    }
    const int waiting = want && !run;
    if (waiting) lu_waited++;
    else fresh_newton = 0;

    // ---------------- C: right-hand side ----------------
    const int active =
        (phase == PH_F0 || phase == PH_F1 || phase == PH_NEWTON) && !nfail && !have_f;
    int okf = 1;
    if (active) {
      okf = rhs();
      cnt[CNT_RHS]++;
    }
    // what the RHS is used for now: not by a waiting cell, which keeps it
    // for its factorization; a cell whose factorization ran takes the F it
    // kept
    int proceed = active && !waiting;
    if (waiting && active) have_f = okf ? 1 : 2;
    if (fac && have_f) {
      proceed = 1;
      okf = have_f == 1;
      have_f = 0;
    }

    // ---------------- D: what the new right-hand side is used for ----------------
    if (proceed) {
      if (phase == PH_F0) {
        if (!okf) {
          status = ST_NONFINITE;
          phase = PH_DONE;
        } else {
          // y0 -> D_0, f0 -> D_1 (scaled by h later); initial step size
          double isc[NS];
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            Dref(0, s) = yv[s];
            Dref(1, s) = F[s];
            isc[s] = 1.0 / (atol + rtol * fabs(yv[s]));
            Dref(ROW_ISC, s) = isc[s];
          }
          const double d0 = wrms(yv, isc);
          d1 = wrms(F, isc);
          h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
          if (h0 > t_end) h0 = t_end;
#pragma unroll
          for (int s = 0; s < NS; ++s) yv[s] = yv[s] + h0 * F[s];
          phase = PH_F1;
        }
      } else if (phase == PH_F1) {
        double df[NS], isc[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          df[s] = F[s] - Dref(1, s);
          isc[s] = Dref(ROW_ISC, s);
        }
        const double d2 = wrms(df, isc) / h0;
        double h1;
        if (!__builtin_isfinite(d2)) {
          h1 = 1e-3 * h0;
        } else {
          const double dm = d1 > d2 ? d1 : d2;
          if (dm <= 1e-15) {
            h1 = 1e-3 * h0;
            if (h1 < 1e-6) h1 = 1e-6;
          } else {
            h1 = sqrt(0.01 / dm);
          }
        }
        hs = 100.0 * h0;
        if (h1 < hs) hs = h1;
        if (t_end < hs) hs = t_end;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          Dref(1, s) = hs * Dref(1, s);
#pragma unroll
          for (int j = 2; j < DROWS; ++j) Dref(j, s) = 0.0;
        }
        cnt[CNT_JAC]++;
        jac_cur = 1;
        jr_ok = 0;
        yj_pred = 0;
        first_jac = 1;
        lu_ok = 0;
        k = 1;
        t = 0.0;
        n_eq = 0;
        need_attempt = 1;
        new_step = 1;
        write_state = 1;
        phase = PH_NEWTON;
      } else {  // PH_NEWTON: one modified-Newton iteration
        int fail = !okf;
        int converged = 0;
        if (!fail) {
          double tmp[NS], isc[NS];
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            tmp[s] = cc * F[s] - Dref(ROW_PSI, s) - dd(s);
            isc[s] = Dref(ROW_ISC, s);
          }
          solve(tmp);
          cnt[CNT_SOLVE]++;
          const double dn = wrms(tmp, isc);
          if (!__builtin_isfinite(dn)) {
            fail = 1;
          } else {
            double rate = 0.0;
            if (it > 0) {
              rate = dn / dprev;
              // predicted error after the remaining iterations,
              // rate^(4 - it) dn / (1 - rate) > tol, with 1 - rate > 0
              // multiplied out
              const double r2 = rate * rate;
              const double rp = it == 1 ? r2 * rate : (it == 2 ? r2 : rate);
              if (rate >= 1.0 || rp * dn > kNewtonTol * (1.0 - rate)) fail = 1;
            }
            if (!fail) {
#pragma unroll
              for (int s = 0; s < NS; ++s) {
                yv[s] += tmp[s];
                dd(s) += tmp[s];
              }
              if (dn == 0.0 || (it > 0 && rate * dn < kNewtonTol * (1.0 - rate))) {
                converged = 1;
              } else {
                dprev = dn;
                it++;
                if (it >= kNewtonMaxIt) fail = 1;
              }
            }
          }
        }
        if (fail) {
          nfail = 1;
        } else if (converged) {
          // error test, scale atol + rtol * max(|y_n|, |y_new|)
          double e1[NS], isc[NS];
          const double rk1 = recip[k + 1];
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const double aa = fabs(Dref(0, s)), bb = fabs(yv[s]);
            isc[s] = rcp_nr(atol + rtol * (aa > bb ? aa : bb));
            e1[s] = divq(dd(s), (double)(k + 1), rk1);
          }
          // err = sqrt(ms) is the error norm; the test err > 1 is taken
          // exactly on ms (the correctly rounded square root exceeds 1
          // exactly when ms exceeds 1 + 2^-52), and log err as (log ms) / 2
          const double ms = wms(e1, isc);
          if (ms > 0x1.0000000000001p+0) {
            double fct = kSafety * exp(0.5 * bn::bn_log(ms) * -rk1);
            if (fct < kMinFactor) fct = kMinFactor;
            hs *= fct;
            pend = fct;
            n_eq = 0;
            lu_ok = 0;
            cnt[CNT_REJ]++;
            need_attempt = 1;
          } else {
            // accept: D_{k+2} = d - D_{k+1}, D_{k+1} = d, D_j += D_{j+1}
            t = t_new;
            double em_acc = 0.0, ep_acc = 0.0;
            const double rk = recip[k], rk2 = recip[k + 2];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
              double dr[KMAX + 1];
#pragma unroll
              for (int j = 0; j <= KMAX; ++j) dr[j] = Dref(j, s);
              const double dk2 = dd(s) - Dref(k + 1, s);
              Dref(k + 1, s) = dd(s);
              double up = dd(s);
#pragma unroll
              for (int j = KMAX; j >= 0; --j) {
                if (j <= k) {
                  up = dr[j] + up;
                  Dref(j, s) = up;
                }
              }
              if (real(s)) {
                const double zm = divq(Dref(k, s), (double)k, rk) * isc[s];
                const double zp = divq(dk2, (double)(k + 2), rk2) * isc[s];
                em_acc += zm * zm;
                ep_acc += zp * zp;
              }
            }
            jac_cur = 0;
            n_eq++;
            cnt[CNT_STEPS]++;
            if (n_eq >= k + 1) {
              em_acc = G::sum(em_acc);
              ep_acc = G::sum(ep_acc);
              // mean squares of the neighbouring orders' estimates
              const double em_s =
                  (k > 1) ? divq(em_acc, (double)n, 1.0 / (double)n) : __builtin_inf();
              const double ep_s =
                  (k < KMAX) ? divq(ep_acc, (double)n, 1.0 / (double)n) : __builtin_inf();
              // the factors norm^(-1/(order+1)) of orders k-1, k, k+1,
              // compared by their logarithms (log norm = (log ms) / 2); one
              // exponential for the best
              const double lm = 0.5 * bn::bn_log(em_s) * -rk;
              const double l0 = 0.5 * bn::bn_log(ms) * -rk1;
              const double lp = 0.5 * bn::bn_log(ep_s) * -rk2;
              double best = l0;
              int dk = 0;
              if (lm > best) {
                best = lm;
                dk = -1;
              }
              if (lp > best) {
                best = lp;
                dk = 1;
              }
              k += dk;
              double fct = kSafety * exp(best);
              if (fct > kMaxFactor) fct = kMaxFactor;
              hs *= fct;
              pend = fct;
              n_eq = 0;
              lu_ok = 0;
            }
            need_attempt = 1;
            new_step = 1;
            if (!(t < t_end)) {
              phase = PH_DONE;
              pend = 0.0;
            }
          }
        }
      }
    }
    // Newton failure: refresh a stale Jacobian at the predicted state and
    // retry with the same step, else halve the step.
    if (nfail) {
      cnt[CNT_NFAIL]++;
      if (!jac_cur) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          dd(s) = 0.0;
          yv[s] = pred(s);
        }
        cnt[CNT_JAC]++;
        jac_cur = 1;
        jr_ok = 0;
        yj_pred = 1;
        lu_ok = 0;
        it = 0;
        fresh_newton = 1;
      } else {
        hs *= 0.5;
        n_eq = 0;
        lu_ok = 0;
        need_attempt = 1;
        pend = 0.5;
      }
    }
    if (pend != 0.0 && phase == PH_NEWTON) rescale(k, pend);
  }
}

// The kernel body: rate multipliers (and the coefficient table) into LDS,
// then one wave per SIMD burns cells from the queue.  LDS: the head
// (head_doubles), then per wave the rows of lds_rows, [rows][NS][64].
template <class NET, int LPC>
__device__ __forceinline__ void burn_kernel_body(const GenArgs &a) {
  constexpr int NS = (NET::n + LPC - 1) / LPC;
  constexpr int RB = (NET::R + 7) / 8 * 8;
  constexpr int HEAD = head_doubles(NET::R, LPC);
  // the launch's dynamic LDS (computed by the host) is what this layout uses
  static_assert(lds_bytes(NS, NET::R, LPC) == NET::HOST_LDS, "LDS layout differs from the host's");
  static_assert(NET::RB == RB, "multiplier block size");
  extern __shared__ double smem[];
  for (int r = threadIdx.x; r < RB; r += blockDim.x)
    smem[r] = r < NET::R ? (a.log_mult ? exp(a.log_mult[r]) : 1.0) : 1.0;
  if constexpr (LPC > 1) {
    for (int i = threadIdx.x; i < HEAD - RECIP - RB; i += blockDim.x) smem[RB + i] = NET::ctab[i];
  }
  // 1/j, correctly rounded (IEEE division)
  if (threadIdx.x < RECIP) smem[HEAD - RECIP + threadIdx.x] = threadIdx.x ? 1.0 / (double)threadIdx.x : 0.0;
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  double *Dw = smem + HEAD + (long long)wave * lds_rows(NS, NET::R, LPC) * NS * 64;
  run_cells<NET, LPC>(a, smem, Dw);
}

}  // namespace bng
