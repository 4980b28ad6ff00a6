// burn_body.h -- device code of the FP64 per-cell reaction-network burn for
// CDNA4 (gfx950), shared by the plain and the persistent kernels.
//
// What is computed follows the single-zone burn of the paper (Sec. 2: the
// network right-hand side and analytic Jacobian generated per network and
// integrated with a VODE-class BDF with self-heating; Sec. 3 runs it zone by
// zone).  The integrator is a variable-order (1..5) BDF in backward
// differences with modified Newton and a dense partially pivoted LU of
// I - cJ (Shampine & Reichelt's quasi-constant step scheme, kappa = 0).  All
// arithmetic is FP64.
//
// Mapping onto a 64-wide wavefront:
//  * Group layout.  A cell is owned by a group of L lanes; component i of
//    its system (species, then temperature, then zero padding up to
//    NP = L*S) lives on lane i % L, slot i / L.  The lanes keep the Newton
//    vectors and the rows of the LU factors (in pivot order) in registers;
//    the backward-difference history D lives in LDS.  The right-hand side
//    spreads the reactions over the group; the triangular solves broadcast
//    one solution component per step inside the group.
//  * Factor layout.  A new LU is needed only every few steps per cell, but
//    with 64/L cells per wave almost every loop iteration has some cell that
//    needs one.  The cells that need a factorization are therefore batched
//    into a wave-wide pass in which every cell gets FL = NP lanes, one matrix
//    row per lane: the Newton matrix is accumulated in LDS from the
//    reaction-parallel Jacobian terms, the LU runs with row-position
//    tracking (no data swaps), and the factors go back to the owning group.
//    One-slot shapes of up to 16 lanes eliminate in the owners' registers
//    and keep J between passes; a lone request waits a few iterations for
//    other cells to need an LU too, since a pass costs the same for one cell
//    as for all.
//  * Control.  Each loop iteration does, per cell: (0) output of a finished
//    cell and intake of the next, (A) step-attempt setup, (B) the wave-wide
//    factorization pass, (C) one right-hand side, (D) the Newton /
//    error-test / step-control logic.  Every heavy routine has one call site,
//    so cells in different phases still share the RHS and solve instructions.
#pragma once

#include "bn_math.h"
#include "burn_internal.h"

#include <math.h>

namespace bn {
namespace {

// pointers into device global memory (address space 1): the accesses through
// them are global, not flat, instructions
typedef __attribute__((address_space(1))) double *gdptr;
typedef const __attribute__((address_space(1))) double *gcdptr;
typedef __attribute__((address_space(1))) int32_t *giptr;

constexpr double kSafety = 0.9;
constexpr double kMinFactor = 0.2;
constexpr double kMaxFactor = 10.0;
constexpr double kNewtonTol = 0.03;
constexpr int kNewtonMaxIt = 4;
constexpr int kMaxDefer = 16;  // iterations an LU request may wait for company

// per-cell phases: the two initial-step RHS, Newton iterations, finished
// (outputs pending), waiting for a cell, no more cells
enum { PH_F0 = 0, PH_F1 = 1, PH_NEWTON = 2, PH_DONE = 3, PH_LOAD = 4, PH_IDLE = 5 };
enum { ST_OK = 0, ST_MAX_STEPS = 1, ST_UNDERFLOW = 2, ST_NONFINITE = 3, ST_BAD_INPUT = 4 };
enum { CNT_STEPS = 0, CNT_REJ, CNT_NFAIL, CNT_RHS, CNT_JAC, CNT_LU, CNT_SOLVE, CNT_ORDER };

// gamma_k = sum_{j=1..k} 1/j, summed in ascending j.
constexpr double gamma_of(int k) {
  double g = 0.0;
  for (int j = 1; j <= k; ++j) g += 1.0 / (double)j;
  return g;
}

// U = R(1) of the step-change transform: U[i][j] = prod_{m=1..i} (m-1-j)/m
// (upper triangular).
constexpr double u_of(int i, int j) {
  double v = 1.0;
  for (int m = 1; m <= i; ++m) v *= (double)(m - 1 - j) / (double)m;
  return v;
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- cross-lane operations inside an aligned group of G lanes --------------

// DPP moves with bound_ctrl set: a lane whose source lane is inactive reads
// 0 (every control used here addresses a lane of the same row), so no old
// value has to be materialised in the destination first.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
  const long long r = ((long long)(unsigned)lo) | ((long long)hi << 32);
  return __builtin_bit_cast(double, r);
}

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

__device__ __forceinline__ double readlane_f64(double v, int src) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __builtin_bit_cast(double, ((long long)(unsigned)lo) | ((long long)hi << 32));
}

// broadcast lane SRC (static) of each aligned group of G lanes
template <int G, int SRC>
__device__ __forceinline__ double gbcast(double v) {
  if constexpr (G == 1) {
    return v;
  } else if constexpr (G == 4) {
    return dpp_f64<SRC | (SRC << 2) | (SRC << 4) | (SRC << 6)>(v);
  } else if constexpr (G == 16) {
    return dpp_f64<0x150 + SRC>(v);  // row_newbcast: lane SRC of each row
  } else if constexpr (G == 8) {
    const double a = dpp_f64<0x150 + SRC>(v), b = dpp_f64<0x150 + 8 + SRC>(v);
    return (threadIdx.x & 8) ? b : a;
  } else if constexpr (G == 64) {
    return readlane_f64(v, SRC);
  } else if constexpr (G == 32) {
    const double lo = readlane_f64(v, SRC), hi = readlane_f64(v, SRC + 32);
    return (__lane_id() & 32) ? hi : lo;
  } else {
    return __shfl(v, SRC, G);
  }
}

// Reduction levels of an aligned group of G lanes.  Each level pairs every
// lane with another (an involution), and after all levels every lane has
// combined all G values (see xch).
template <int G>
constexpr int n_levels() {
  return G >= 64 ? 6 : G >= 32 ? 5 : G >= 16 ? 4 : G >= 8 ? 3 : G >= 4 ? 2 : G >= 2 ? 1 : 0;
}

// Exchange with the lane 16 (32) apart: gfx950's permlane16 (permlane32)
// swap of a register with itself leaves the even and odd rows (the two
// halves) in its two results; each lane takes its partner's.
__device__ __forceinline__ int xor16_i32(int v) {
  const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return (threadIdx.x & 16) ? r[0] : r[1];
}
__device__ __forceinline__ int xor32_i32(int v) {
  const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return (threadIdx.x & 32) ? r[0] : r[1];
}
__device__ __forceinline__ double xor16_f64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = xor16_i32((int)(b & 0xffffffffLL)), hi = xor16_i32((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)(unsigned)lo) | ((long long)hi << 32));
}
__device__ __forceinline__ double xor32_f64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = xor32_i32((int)(b & 0xffffffffLL)), hi = xor32_i32((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)(unsigned)lo) | ((long long)hi << 32));
}

// Level LV of a G-lane reduction: from the last level backwards, xor 1 and
// xor 2 (DPP quad permutes), the half-row and row mirrors (DPP), then xor 16
// and xor 32 (permlane swaps).  All stay in VALU.
template <int G, int LV>
__device__ __forceinline__ double xch(double v) {
  constexpr int NL = n_levels<G>();
  constexpr int FROM_END = NL - 1 - LV;
  if constexpr (FROM_END == 0) return dpp_f64<0xB1>(v);
  else if constexpr (FROM_END == 1) return dpp_f64<0x4E>(v);
  else if constexpr (FROM_END == 2) return dpp_f64<0x141>(v);
  else if constexpr (FROM_END == 3) return dpp_f64<0x140>(v);
  else if constexpr (FROM_END == 4) return xor16_f64(v);
  else return xor32_f64(v);
}

template <int G, int LV>
__device__ __forceinline__ int xch_i(int v) {
  constexpr int NL = n_levels<G>();
  constexpr int FROM_END = NL - 1 - LV;
  if constexpr (FROM_END == 0) return dpp_i32<0xB1>(v);
  else if constexpr (FROM_END == 1) return dpp_i32<0x4E>(v);
  else if constexpr (FROM_END == 2) return dpp_i32<0x141>(v);
  else if constexpr (FROM_END == 3) return dpp_i32<0x140>(v);
  else if constexpr (FROM_END == 4) return xor16_i32(v);
  else return xor32_i32(v);
}

// All-reduce sum; every lane ends with the bitwise same value because each
// level adds two partial sums that are equal up to commutation.
template <int G, int LV = 0>
__device__ __forceinline__ double gsum(double v) {
  if constexpr (LV < n_levels<G>()) {
    v += xch<G, LV>(v);
    return gsum<G, LV + 1>(v);
  } else {
    return v;
  }
}

// Any of the group's active lanes nonzero (1 or 0): one ballot and the
// group's bits of it, instead of a chain of exchanges.
template <int G>
__device__ __forceinline__ int gor(int v) {
  const unsigned long long m = __ballot(v != 0);
  if constexpr (G >= 64) {
    return m != 0ULL;
  } else {
    const int base = (int)(threadIdx.x & 63) & ~(G - 1);
    return ((m >> base) & ((1ULL << G) - 1)) != 0ULL;
  }
}

// Calls f.template operator()<I>() for I = 0..N-1 (compile-time indices).
template <int N>
struct Unroll {
  template <typename F>
  __device__ __forceinline__ static void run(F &&f) {
    Unroll<N - 1>::run(f);
    f.template operator()<N - 1>();
  }
};
template <>
struct Unroll<0> {
  template <typename F>
  __device__ __forceinline__ static void run(F &&) {}
};

// Arg-max of v over the group, ties to the smallest key: the maximum of v
// first (NaN-free inputs), then the smallest key among the lanes that hold
// it.  Two plain reductions instead of a lexicographic compare per level.
template <int G>
__device__ __forceinline__ void gargmax_key(double &v, int &key) {
  double m = v;
  Unroll<n_levels<G>()>::run([&]<int LV>() __attribute__((always_inline)) {
    m = fmax(m, xch<G, LV>(m));
  });
  int k = (v == m) ? key : 0x7fffffff;
  Unroll<n_levels<G>()>::run([&]<int LV>() __attribute__((always_inline)) {
    k = min(k, xch_i<G, LV>(k));
  });
  v = m;
  key = k;
}



// ---------------------------------------------------------------------------
// LDS layout.  Per workgroup, the network tables (every array starts on a
// 16-byte boundary, so a reaction's output list is one aligned 16-byte pair):
//   rtab[8 Rb] (doubles, Rb = R rounded up to 32; see coef_of) | rout[8R] rsp[4R] (ints)
//   | emult[R] q[R] qcv[R] (doubles) | recip[8] (1/j for j = 0..7, entry 0 unused)
// then one area per wave:
//   D[CPW][DS] ybuf[CPW][YS] facc[CPW][YS] fslot[FC][FB] fsc[FC][4]
// with FB = NP + n*MS + 2*NP + 1 doubles per factorization slot: y_J, the
// Newton matrix (n rows, odd row stride MS, later the factors in place) and
// two auxiliary rows (reciprocal pivots and row indices by position).  The
// per-cell strides DS and YS place the cells of a half-wave on disjoint LDS
// banks (see Shape) and MS is odd, so the rows of a matrix fall in
// different banks.
// ---------------------------------------------------------------------------

// The rate coefficients are stored in blocks of 32 reactions, coefficient
// by coefficient: reaction r = 32a + b has coefficient k at
// ((8a + k) * 32 + b).  Lanes working on consecutive reactions then read
// consecutive doubles (no bank conflicts), and the eight coefficients of a
// reaction sit at constant offsets from its first.
__host__ __device__ inline size_t rblk_of(int R) { return ((size_t)R + 31) & ~(size_t)31; }
__host__ __device__ inline size_t tab_doubles_of(int R) { return 8 * rblk_of(R) + 9 * (size_t)R + 8; }

// coefficient k of one reaction: c[k]
struct Coef {
  const double *p;
  __device__ __forceinline__ double operator[](int k) const { return p[32 * k]; }
};
__device__ __forceinline__ Coef coef_of(const double *rtab, int r) {
  return Coef{rtab + ((size_t)(r >> 5) * 256 + (r & 31))};
}

template <int L, int S>
struct Shape {
  static constexpr int NP = L * S;
  // Small systems keep all NP rows with the compile-time stride NP + 1 (the
  // padded rows are identity rows); large ones store only the n real rows
  // with the odd stride n | 1, which keeps a 51-component matrix in 21 KB.
  static constexpr bool COMPACT = NP >= 32;
  __host__ __device__ static int ms(int n) { return COMPACT ? (n | 1) : NP + 1; }
  __host__ __device__ static int rows(int n) { return COMPACT ? n : NP; }
  static constexpr int CPW = 64 / L;
  static constexpr int FL = NP;       // factor lanes per cell (one row each)
  static constexpr int FC = 64 / NP;  // cells per factorization pass
  static constexpr int ECH = NP >= 64 ? 8 : 4;  // elimination columns per LDS batch
  static_assert(NP == 4 || NP == 8 || NP == 16 || NP == 32 || NP == 64, "NP must be a power of 2");
  // Per-cell strides.  A wave's LDS access is served half a wave (32 lanes)
  // at a time; the 32/L cells of a half-wave each touch 2L consecutive banks
  // (L consecutive doubles).  A cell stride that is an odd multiple of L
  // doubles puts them on disjoint banks.  Groups of 32 or 64 lanes fill a
  // half-wave alone.
  static constexpr int stride_for(int base) {
    if (L >= 32) return base + 4;
    const int m = (base + L - 1) / L;
    return (m % 2 ? m : m + 1) * L;
  }
  static constexpr int DS = stride_for(DROWS * NP);  // history stride per cell
  static constexpr int YS = stride_for(NP);          // exchange-vector stride per cell
  __host__ __device__ static size_t fb(int n) {
    return (size_t)NP + (size_t)rows(n) * ms(n) + 2 * (size_t)NP + 1;
  }
  __host__ __device__ static size_t wave_doubles(int n) {
    return (size_t)CPW * DS + 2 * (size_t)CPW * YS + FC * fb(n) + 4 * FC;
  }
};

struct Tabs {
  const double *rtab, *emult, *q, *qcv, *recip;
  const int *rsp, *rout;
};

// Entry E (0..5) of a reaction's species list (rout row ro0, ro1).  Past the
// reaction's own count the table holds coefficient-0 entries on its first
// listed species, so that all lanes of a wave take the same number of
// entries (the network's largest count) without a branch or a select per
// entry.  A padded entry adds w x = +-0, which leaves the accumulator
// unchanged (an accumulator that starts at +0 never holds -0), or NaN when x
// is not finite; x is then a rate or a rate derivative of the same reaction,
// and that reaction's heat term (q x) or the caller's finiteness check
// already marks the evaluation as failed.
struct Ent {
  int sp;    // species
  double w;  // nu_ir, or 0 for a padded entry
};
template <int E>
__device__ __forceinline__ Ent ent_of(const int4 &ro0, const int4 &ro1) {
  static_assert(E >= 0 && E < 6, "a reaction changes at most 6 species");
  const int raw = E == 0   ? ro0.y
                  : E == 1 ? ro0.z
                  : E == 2 ? ro0.w
                  : E == 3 ? ro1.x
                  : E == 4 ? ro1.y
                           : ro1.z;
  Ent r;
  r.sp = raw >> 8;
  r.w = (double)(int)(signed char)(raw & 0xff);
  return r;
}

__device__ __forceinline__ Tabs tabs_at(double *smem, int R) {
  Tabs t;
  t.rtab = smem;
  t.rout = reinterpret_cast<const int *>(smem + 8 * rblk_of(R));
  t.rsp = t.rout + 8 * R;
  t.emult = reinterpret_cast<const double *>(t.rsp + 4 * R);
  t.q = t.emult + R;
  t.qcv = t.q + R;
  t.recip = t.qcv + R;
  return t;
}

// Copy a network's tables into LDS (all threads of the workgroup take part;
// the caller synchronizes).
__device__ __forceinline__ void load_tables(const NetTables &nt, const double *log_mult,
                                            double *smem) {
  const int R = nt.R;
  double *rtab = smem;
  int *rout = reinterpret_cast<int *>(smem + 8 * rblk_of(R));
  int *rsp = rout + 8 * R;
  double *emult = reinterpret_cast<double *>(rsp + 4 * R);
  double *q = emult + R;
  double *qcv = q + R;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int i = tid; i < 8 * R; i += nth) {
    const int r = i >> 3, k = i & 7;
    rtab[((r >> 5) * 8 + k) * 32 + (r & 31)] = nt.rtab[i];
    rout[i] = nt.rout[i];
  }
  for (int i = tid; i < R; i += nth) {
    emult[i] = log_mult ? exp(log_mult[i]) : 1.0;
    q[i] = nt.q[i];
    qcv[i] = nt.q[i] * nt.inv_cv;
  }
  for (int i = tid; i < 4 * R; i += nth) rsp[i] = nt.rsp[i];
  // 1/j, correctly rounded (IEEE division): the step controller's
  // order-dependent quotients read these instead of dividing
  if (tid < 8) qcv[R + tid] = tid ? 1.0 / (double)tid : 0.0;
}

// Burn cells with one wave.  The cells come either from a static map (cell
// first_cell for this lane group, then nothing) or, when queue is not null,
// from a device work queue: a group whose cell has finished writes it out and
// takes the next index from the queue, until the queue passes n_cells.  The
// loop ends when every group of the wave is idle.  With REC the accepted
// steps' schedule (order, step size, product of the history rescale ratios
// since the previous accepted step) is recorded for a sensitivity replay.
// With SRC a constant per-cell source is added to the right-hand side.  With
// SCR every rate carries the synthetic screening factor exp(h_r G),
// G = sqrt(rho (1 + sum_j A_j^2 Y_j)) T^(-3/2), and the Jacobian its terms
// (a rank-one composition part u_i dG/dY_j and dG/dT in the T column).
// With PROBE a cell stops after the initial step size h0 and writes only
// h0 to a.key (the queue order of the persistent kernel).
template <int L, int S, bool QUEUE, bool REC = false, bool SRC = false, bool SCR = false,
          bool PROBE = false>
__device__ __forceinline__ void run_cells(const BurnArgs &a, const Tabs &tb, double *wb,
                                          int64_t first_cell, unsigned long long *queue) {
  static_assert(!(PROBE && (QUEUE || REC)), "the order probe runs on the static map alone");
  using SH = Shape<L, S>;
  constexpr int NP = SH::NP, CPW = SH::CPW, FL = SH::FL, FC = SH::FC;
  constexpr int DS = SH::DS, YS = SH::YS, ECH = SH::ECH;
  // one-slot shapes (a cell per group, NP = L) factor in registers
  constexpr bool REG_LU = S == 1 && NP <= 16;

  const NetTables &nt = a.net;
  const int N = nt.N, R = nt.R;
  const int ne = nt.max_ent;  // entries per reaction, padded (ent_of)
  int n = nt.n;  // re-derived opaquely in every iteration, like q
  const int MS = SH::ms(n);
  // the norms' mean over the n components, sum / n, without a division
  const double dn_sz = (double)n, inv_n = 1.0 / dn_sz;
  const int MROWS = SH::rows(n);
  const size_t FB = SH::fb(n);

  const int lane = threadIdx.x & 63;
  int q = lane % L;  // re-derived opaquely in every iteration (see below)
  const int cw = lane / L;
  // Launch constants used inside the cell loop.  Each is made opaque once,
  // so it lives in scalar registers of its own: loaded as part of one wide
  // kernel-argument load, a value would otherwise tie the whole load's
  // registers together, and a spill of it reloads all of them.
  int64_t C = a.n_cells;
  double rtol = a.rtol, atol = a.atol, t_end = a.t_end;
  // (global, not flat, pointers: a flat access also counts as an LDS
  // access, so an LDS wait after a flat store would wait for the store)
  gdptr gY = (gdptr)a.Y, gT = (gdptr)a.T;
  gcdptr grho = (gcdptr)a.rho;
  giptr gst = (giptr)a.status, gcnt = (giptr)a.counters;
  int max_steps = a.max_steps;
  asm volatile("" : "+s"(C), "+s"(rtol), "+s"(atol), "+s"(t_end));
  asm volatile("" : "+s"(gY), "+s"(gT), "+s"(grho), "+s"(gst), "+s"(gcnt), "+s"(max_steps));

  double *Dl = wb + (size_t)cw * DS;  // this cell's history, [DROWS][NP]
  double *ybuf = wb + (size_t)CPW * DS + (size_t)cw * YS;
  double *facc = wb + (size_t)CPW * DS + (size_t)CPW * YS + (size_t)cw * YS;
  double *fbase = wb + (size_t)CPW * DS + 2 * (size_t)CPW * YS;
  double *fsc = fbase + (size_t)FC * FB;
  // this wave's Jacobian areas (shapes that factor in LDS, when the launch
  // provides them): cell c of the wave keeps J(y_J) at jw + c MROWS^2,
  // column-major
  gdptr jw = nullptr;
  if constexpr (!REG_LU) {
    if (a.jws) {
      const int wv = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
      jw = (gdptr)a.jws + (size_t)wv * (size_t)a.jws_wave;
    }
  }

  const double *s_rtab = tb.rtab, *s_emult = tb.emult, *s_q = tb.q, *s_qcv = tb.qcv;
  const double *s_recip = tb.recip;
  const int *s_rsp = tb.rsp, *s_rout = tb.rout;

  // ---- per-lane state (group layout)
  double LU[S][NP];  // factor rows held at positions s*L+q
  // register factorization: row q of the cell's J(y_J), kept between passes
  double Jr[REG_LU ? NP : 1];
  int jr_ok = 0;  // J(y_J) is held (in Jr, or in the cell's workspace area)
  double dinv[S];    // 1 / U_pp of those rows
  int ridx[S];       // natural index of those rows
  double yp[S], psi[S], isc[S], dd[S], yv[S], yJ[S], F[S];
  double srcv[S];  // constant source of the own components (SRC)
  double wsqv[S];  // A_i^2 of the own species components (SCR)
#pragma unroll
  for (int s = 0; s < S; ++s) {
    dinv[s] = 1.0;
    ridx[s] = s * L + q;
#pragma unroll
    for (int j = 0; j < NP; ++j) LU[s][j] = 0.0;
    yp[s] = psi[s] = isc[s] = dd[s] = yv[s] = yJ[s] = F[s] = srcv[s] = 0.0;
    wsqv[s] = 0.0;
    if constexpr (SCR) {
      if (s * L + q < nt.N) wsqv[s] = nt.wsq[s * L + q];
    }
  }
#pragma unroll
  for (int j = 0; j < (REG_LU ? NP : 1); ++j) Jr[j] = 0.0;
  int cnt[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) cnt[c] = 0;

  auto comp = [&](int s) __attribute__((always_inline)) { return s * L + q; };

  // weighted RMS norm over the n real components (inv = 1/scale)
  auto wrms = [&](const double(&v)[S], const double(&inv)[S]) __attribute__((always_inline)) {
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const double z = v[s] * inv[s];
      if (comp(s) < n) acc += z * z;
    }
    return sqrt(bn_div_by(gsum<L>(acc), dn_sz, inv_n));
  };

  // change of step size by ratio rh on rows 0..k of D: D <- (R(rh) U)^T D,
  // applied in its two factors (values at the new nodes, then differences)
  double racc = 1.0;  // rescale ratios since the last accepted step (REC)
  auto rescale = [&](int k, double rh) __attribute__((always_inline)) {
    if constexpr (REC) racc *= rh;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = comp(s);
      double dcol[KMAX + 1];
#pragma unroll
      for (int b = 0; b <= KMAX; ++b) {
        const double x = Dl[b * NP + i];  // read unconditionally, used for b <= k
        dcol[b] = (b <= k) ? x : 0.0;
      }
      // rows b > k are zero in dcol, so their terms add exactly nothing; the
      // node m = 0 reproduces D_0; entries aa <= k use only m <= aa <= k
      double v[KMAX + 1];
      v[0] = dcol[0];
#pragma unroll
      for (int m = 1; m <= KMAX; ++m) {
        const double x = (double)m * rh;
        double rb = 1.0;
        double acc = dcol[0];
#pragma unroll
        for (int b = 1; b <= KMAX; ++b) {
          rb *= ((double)(b - 1) - x) * (1.0 / (double)b);
          acc += rb * dcol[b];
        }
        v[m] = acc;
      }
#pragma unroll
      for (int aa = 0; aa <= KMAX; ++aa) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m <= aa; ++m) acc += u_of(m, aa) * v[m];
        if (aa <= k) Dl[aa * NP + i] = acc;
      }
    }
  };

  double rho = 1.0;

  // ---- right-hand side F = f(yv) for the own components; 1 if finite.
  // The group's lanes take the reactions r = q, q+L, ...; each rate is added
  // into the accumulator of every species it changes with LDS atomics, one
  // instruction per entry slot of the reactions' species lists.  A species'
  // terms are therefore summed slot by slot (every reaction for which it is
  // the first listed species, then the second, ...), within a slot in lane
  // order: not the ascending reaction order of the definition, so the sums
  // round differently from a serial sum.  The heat term is a tree sum over
  // the group's lanes times 1/c_v.
  auto rhs = [&]() __attribute__((always_inline)) -> int {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      ybuf[comp(s)] = yv[s];
      facc[comp(s)] = 0.0;
    }
    wave_lds_sync();
    const double T = ybuf[N];
    const double t13 = cbrt(T);
    const double tinv = 1.0 / T;
    const double tm13 = (t13 * t13) * tinv;  // T^(-1/3) = T^(2/3) / T
    const double t53 = T * t13 * t13;
    const double lnT = bn_log(T);
    double G = 0.0;
    if constexpr (SCR) {
      double part = 0.0;
#pragma unroll
      for (int s = 0; s < S; ++s) part += wsqv[s] * yv[s];
      G = sqrt(rho * (1.0 + gsum<L>(part))) / (T * sqrt(T));
    }
    double heat = 0.0;
    auto one = [&](int r) __attribute__((always_inline)) {
      const Coef c = coef_of(s_rtab, r);
      double expo =
          c[0] + c[1] * tinv + c[2] * tm13 + c[3] * t13 + c[4] * T + c[5] * t53 + c[6] * lnT;
      if constexpr (SCR) expo += nt.screen[r] * G;
      // reactant slots: all loads issued unconditionally (an absent slot
      // reads entry 0 and multiplies by 1), so they overlap the exponential
      const int4 sp = *reinterpret_cast<const int4 *>(s_rsp + 4 * r);
      const double ya = ybuf[sp.x < 0 ? 0 : sp.x];
      const double yb = ybuf[sp.y < 0 ? 0 : sp.y];
      const double yc = ybuf[sp.z < 0 ? 0 : sp.z];
      double v = exp(expo) * s_emult[r] * c[7];
      // rho^(n_r - 1) for n_r <= 3 reactants
      if (sp.w >= 2) v *= rho;
      if (sp.w >= 3) v *= rho;
      v *= (sp.x >= 0 ? ya : 1.0);
      v *= (sp.y >= 0 ? yb : 1.0);
      v *= (sp.z >= 0 ? yc : 1.0);
      heat += s_q[r] * v;
      const int4 *ro = reinterpret_cast<const int4 *>(s_rout + 8 * r);
      const int4 r0 = ro[0], r1 = ro[1];
      Unroll<6>::run([&]<int E>() __attribute__((always_inline)) {
        if (E < ne) {
          const Ent en = ent_of<E>(r0, r1);
          __hip_atomic_fetch_add(&facc[en.sp], en.w * v, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
      });
    };
    for (int r = q; r < R; r += 2 * L) {
      one(r);
      if (r + L < R) one(r + L);
    }
    heat = gsum<L>(heat);
    wave_lds_sync();
    int bad = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = comp(s);
      double f = (i < N) ? facc[i] : ((i == N) ? heat * nt.inv_cv : 0.0);
      if constexpr (SRC) f = f + srcv[s];
      F[s] = f;
      if (i < n && !isfinite(f)) bad = 1;
    }
    return !gor<L>(bad);
  };

  // ---- M x = b with the factors (b natural order in, x natural order out)
  auto solve = [&](double(&b)[S]) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < S; ++s) ybuf[comp(s)] = b[s];
    wave_lds_sync();
#pragma unroll
    for (int s = 0; s < S; ++s) {
      b[s] = ybuf[ridx[s]];
      if constexpr (SH::COMPACT) b[s] = comp(s) < n ? b[s] : 0.0;
    }
    // forward substitution with the unit lower factor.  Positions K >= n
    // are padding (zero right-hand side, zero factor rows and columns, unit
    // diagonal): they change nothing, so the compact layout skips the
    // blocks of eight columns that lie wholly past n (one test per block;
    // the padded columns of the last block run and add zeros).
    // (n is made opaque before each sweep, so the block tests are not kept
    // from one sweep to the other)
    constexpr int SB = NP < 8 ? NP : 8;  // columns per skip test
    static_assert(NP % SB == 0, "whole blocks of columns");
    int nf = n;
    asm volatile("" : "+s"(nf));
    Unroll<NP / SB>::run([&]<int BK>() __attribute__((always_inline)) {
      if (!SH::COMPACT || BK * SB < nf) {
        Unroll<SB>::run([&]<int KI>() __attribute__((always_inline)) {
          constexpr int K = BK * SB + KI;
          const double xk = gbcast<L, K % L>(b[K / L]);
          // the factor column masked to the strictly lower part (a select
          // that does not wait for xk) and an unconditional update: b - 0 xk
          // is b
#pragma unroll
          for (int s = K / L; s < S; ++s) {
            const double lk = comp(s) > K ? LU[s][K] : 0.0;
            b[s] = fma(-lk, xk, b[s]);
          }
        });
      }
    });
    // back substitution with the upper factor: at step K component K is
    // final, x_K = b_K / U_KK goes to the components above it; each lane
    // scales its own components once at the end (the same product)
    int nb = n;
    asm volatile("" : "+s"(nb));
    Unroll<NP / SB>::run([&]<int BB>() __attribute__((always_inline)) {
      constexpr int BK = NP / SB - 1 - BB;
      if (!SH::COMPACT || BK * SB < nb) {
        Unroll<SB>::run([&]<int KI>() __attribute__((always_inline)) {
          constexpr int K = BK * SB + SB - 1 - KI;
          const double xk = gbcast<L, K % L>(b[K / L] * dinv[K / L]);
#pragma unroll
          for (int s = 0; s <= K / L; ++s) {
            const double uk = comp(s) < K ? LU[s][K] : 0.0;  // strictly upper part
            b[s] = fma(-uk, xk, b[s]);
          }
        });
      }
    });
#pragma unroll
    for (int s = 0; s < S; ++s) b[s] = b[s] * dinv[s];
    wave_lds_sync();
  };

  // ================= cell state machine =================
  int64_t cell = -1;
  int phase = PH_LOAD;
  int status = 0, write_state = 0;
  int k = 1, n_eq = 0, jac_cur = 0, lu_ok = 0, it = 0, need_attempt = 0, new_step = 0;
  int fresh_newton = 0, first_jac = 0, defer_it = 0;
  int f_pre = 0, okf_pre = 1;  // F already holds f(predictor), computed while waiting
  float probe_h0 = __builtin_inff();  // PROBE: h0, or +inf for a cell that fails first
  double t = 0.0, h = 0.0, t_new = 0.0, cc = 0.0, dprev = 0.0, err = 0.0, h0 = 0.0, d1 = 0.0;

  // outputs of the group's cell: state (if integration started), status and
  // counters
  auto write_out = [&]() __attribute__((always_inline)) {
    if (write_state) {
      cnt[CNT_ORDER] = k;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int i = comp(s);
        if (i < N) gY[(int64_t)i * C + cell] = Dl[i];
        else if (i == N) gT[cell] = Dl[i];
      }
    }
    if constexpr (REC) {
      if (q == 0)
        a.sched[cell * a.sched_stride] = (status == ST_OK) ? (double)cnt[CNT_STEPS] : -1.0;
    }
    if (q == 0) {
      if (gst) gst[cell] = status;
      if (gcnt) {
#pragma unroll
        for (int c = 0; c < 8; ++c)
          gcnt[(int64_t)c * C + cell] = (status == ST_BAD_INPUT) ? 0 : cnt[c];
      }
    }
  };

  // take cell c (or go idle if c >= C): load its state and check the inputs
  auto load_cell = [&](int64_t c) __attribute__((always_inline)) {
    if (c >= C) {
      phase = PH_IDLE;
      return;
    }
    cell = c;
    rho = grho[cell];
    status = 0;
    write_state = 0;
    f_pre = 0;
    k = 1;
    n_eq = jac_cur = lu_ok = it = need_attempt = new_step = fresh_newton = first_jac = 0;
    t = h = t_new = cc = dprev = err = h0 = d1 = 0.0;
#pragma unroll
    for (int c8 = 0; c8 < 8; ++c8) cnt[c8] = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = comp(s);
      yv[s] = (i < N) ? gY[(int64_t)i * C + cell] : ((i == N) ? gT[cell] : 0.0);
      if constexpr (SRC) srcv[s] = (i < n) ? a.src[(int64_t)i * C + cell] : 0.0;
    }
    int bad = !(rho > 0.0) || !isfinite(rho);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = comp(s);
      if (i < n && !isfinite(yv[s])) bad = 1;
      if (i == N && !(yv[s] > 0.0)) bad = 1;
      if constexpr (SRC) {
        if (i < n && !isfinite(srcv[s])) bad = 1;
      }
    }
    if (gor<L>(bad)) {
      status = ST_BAD_INPUT;
      phase = PH_DONE;
    } else {
      phase = PH_F0;
    }
  };
  if constexpr (!QUEUE) load_cell(first_cell);

  while (true) {
    // The lane index is made opaque to the compiler once per iteration, so
    // the many lane predicates of the unrolled loops (q > K, q == K, ...) are
    // computed where they are used instead of being hoisted out of this loop
    // and kept live as scalar masks, which exceeds the scalar registers and
    // spills them.  The same holds for the uniform tests K < n.
    asm volatile("" : "+v"(q));
    asm volatile("" : "+s"(n));
    // ---------------- 0: write a finished cell, take the next one ----------------
    if constexpr (QUEUE) {
      if (phase == PH_DONE) {
        write_out();
        phase = PH_LOAD;
      }
    }
    if constexpr (QUEUE) {
      const unsigned long long lmask = __ballot(phase == PH_LOAD && q == 0);
      if (lmask && a.parts) {
        // ordered launch: positions of this workgroup's XCD first (cells
        // that run on one XCD then share its L2 lines), then the other parts;
        // at most XCD_PARTS atomics per group, then the group is idle
        if (phase == PH_LOAD) {
          long long got = -1;
          if (q == 0) {
            const int x0 = (int)(blockIdx.x % XCD_PARTS);
            const long long per = C / XCD_PARTS, extra = C % XCD_PARTS;
            for (int t = 0; t < XCD_PARTS && got < 0; ++t) {
              const int x = (x0 + t) % XCD_PARTS;
              const long long count = per + (x < extra ? 1 : 0);
              const unsigned long long i = atomicAdd(&a.parts[x], 1ULL);
              if ((long long)i < count) got = x * per + (x < extra ? x : extra) + (long long)i;
            }
          }
          got = __builtin_bit_cast(long long, gbcast<L, 0>(__builtin_bit_cast(double, got)));
          load_cell(got >= 0 && got < C ? (int64_t)got : C);
        }
      } else if (lmask) {
        // one atomic per wave; the requesting groups take consecutive indices
        const int leader = __ffsll((long long)lmask) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(queue, (unsigned long long)__popcll(lmask));
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(base & 0xffffffffULL), leader);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(base >> 32), leader);
        base = ((unsigned long long)hi << 32) | lo;
        const unsigned long long below = lmask & ((1ULL << (cw * L)) - 1ULL);
        const unsigned long long idx = base + (unsigned long long)__popcll(below);
        if (phase == PH_LOAD) load_cell(idx < (unsigned long long)C ? (int64_t)idx : C);
      }
    }
    // static map: a finished cell stays done and is written after the loop
    if (__ballot(phase != PH_IDLE && (QUEUE || phase != PH_DONE)) == 0) break;

    // ---------------- A: start of a step attempt ----------------
    if (phase == PH_NEWTON && need_attempt) {
      if (new_step && cnt[CNT_STEPS] >= max_steps) {
        status = 1;
        phase = PH_DONE;
      } else {
        // step underflow (also catches a non-finite h, so every cell ends)
        // 10 ulp(t) for t >= 0: the next double above t, minus t
        const double ulp =
            __builtin_bit_cast(double, __builtin_bit_cast(long long, t) + 1LL) - t;
        if (!(h >= 10.0 * ulp)) {
          status = 2;
          phase = PH_DONE;
        } else {
          t_new = t + h;
          if (t_new > t_end) {
            t_new = t_end;
            rescale(k, (t_end - t) / h);
            h = t_end - t;
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
          for (int s = 0; s < S; ++s) {
            const int i = comp(s);
            double sa = Dl[i];
            double sb = 0.0;
            // rows 1..KMAX are read whatever k is (rows above k are unused),
            // so no load waits behind a branch on k
            double dr[KMAX + 1];
#pragma unroll
            for (int j = 1; j <= KMAX; ++j) dr[j] = Dl[j * NP + i];
#pragma unroll
            for (int j = 1; j <= KMAX; ++j) {
              if (j <= k) {
                sa += dr[j];
                sb += gamma_of(j) * dr[j];
              }
            }
            yp[s] = sa;
            psi[s] = sb * igk;
            isc[s] = 1.0 / (atol + rtol * fabs(sa));
            dd[s] = 0.0;
            yv[s] = sa;
          }
          cc = h / gk;
          it = 0;
          need_attempt = 0;
          new_step = 0;
          fresh_newton = 1;
        }
      }
    }

    // ---------------- B: LU pass for the cells that need one ----------------
    // A pass costs the same whatever number of its slots are used.  When the
    // wave can factor several cells in one pass, LU requests wait (up to
    // kMaxDefer iterations) until every slot would be used, or every cell
    // that still has work wants one.  A waiting cell does nothing in those
    // iterations (no RHS, no Newton), so its own computation, and its
    // results, are unchanged.
    int want = (phase == PH_NEWTON && fresh_newton && !lu_ok);
    int defer = 0;
    if constexpr (FC >= 2 && CPW >= 2) {
      const unsigned long long wm = __ballot(want && q == 0);
      const unsigned long long expired = __ballot(want && q == 0 && defer_it >= kMaxDefer);
      const int busy =
          __popcll(__ballot((phase == PH_F0 || phase == PH_F1 || phase == PH_NEWTON) && q == 0));
      const int target = busy < FC ? busy : FC;
      if (want && __popcll(wm) < target && !expired) defer = 1;
      defer_it = defer ? defer_it + 1 : 0;
      if (defer) want = 0;
    }
    int sing = 0;
    unsigned long long wmask = __ballot(want && q == 0);
    while (wmask) {
      int sel[FC];
      if constexpr (REG_LU) {
        // one cell per slot (FC == CPW): every cell factors in its own
        // group's lanes, so the rows can stay in the owners' registers
#pragma unroll
        for (int j = 0; j < FC; ++j) sel[j] = ((wmask >> (j * L)) & 1) ? j : -1;
        wmask = 0;
      } else {
#pragma unroll
        for (int j = 0; j < FC; ++j) {
          if (wmask) {
            sel[j] = (__ffsll((long long)wmask) - 1) / L;
            wmask &= wmask - 1;
          } else {
            sel[j] = -1;
          }
        }
      }
      // (a) the selected cells publish y_J, c and rho
      int myslot = -1;
#pragma unroll
      for (int j = 0; j < FC; ++j)
        if (sel[j] == cw) myslot = j;
      if (myslot >= 0) {
        double *py = fbase + (size_t)myslot * FB;
#pragma unroll
        for (int s = 0; s < S; ++s) py[comp(s)] = yJ[s];
        if (q == 0) {
          fsc[4 * myslot + 0] = cc;
          fsc[4 * myslot + 1] = rho;
          // the cell's area holds J(y_J) (read in (b), overwritten in (d))
          fsc[4 * myslot + 2] = (jw && jr_ok) ? 1.0 : 0.0;
        }
      }
      wave_lds_sync();
      // (b) factor layout: slot fj = lane / FL, row fi = lane % FL; in the
      // compact layout the rows fi >= n of a padded system take no part
      int flane = lane;
      asm volatile("" : "+v"(flane));
      const int fj = flane / FL, fi = flane % FL;
      int fsel = -1;
#pragma unroll
      for (int j = 0; j < FC; ++j)
        if (j == fj) fsel = sel[j];
      double *fy = fbase + (size_t)fj * FB;
      double *fM = fy + NP;  // Newton matrix [MROWS][MS], row-major
      const double fcc = fsel >= 0 ? fsc[4 * fj + 0] : 0.0;
      const double frho = fsel >= 0 ? fsc[4 * fj + 1] : 1.0;
      const bool frow = fi < MROWS;
      double *uacc = fM + (size_t)MROWS * MS;  // screening: sum_r W_ir h_r R_r
      // J(y_J) is assembled (into LDS, unscaled, from a zero matrix) only
      // when it was refreshed: with register factorization it is kept in the
      // lanes' Jr registers, otherwise in the cell's area of the workspace
      // (without one, every pass assembles it); the pass then builds I - cJ
      // from it.
      bool asm_j;
      if constexpr (REG_LU) asm_j = fsel >= 0 && !jr_ok;
      else asm_j = fsel >= 0 && !(fsc[4 * fj + 2] != 0.0);
      const bool any_asm = __ballot(asm_j) != 0;
      int jbad = 0;
      if (any_asm) {
      if constexpr (SH::COMPACT) {
        if (frow) {
          if constexpr (SCR) uacc[fi] = 0.0;
          double *mr = fM + fi * MS;
          for (int j = 0; j < MROWS; ++j) mr[j] = 0.0;
        }
      } else {
        // the slot's FL lanes zero its matrix together (consecutive
        // addresses, constant offsets), then each row lane sets its diagonal
#pragma unroll
        for (int i = 0; i < NP * (NP + 1); i += FL) fM[i + fi] = 0.0;
        wave_lds_sync();
        if constexpr (SCR) uacc[fi] = 0.0;
      }
      wave_lds_sync();
      // Rates at y_J for the reactions r = fi, fi+FL, ...; every Jacobian term
      // W(i, r) dR_r/dy_j (W = nu for a species row, q/c_v for the temperature
      // row) is added into J.
      double fG = 0.0, fS = 1.0;
      if (fsel >= 0 && asm_j) {
        const double T = fy[N];
        const double t13 = cbrt(T);
        const double tinv = 1.0 / T;
        const double tm13 = (t13 * t13) * tinv;  // T^(-1/3) = T^(2/3) / T
        const double t53 = T * t13 * t13;
        const double lnT = bn_log(T);
        if constexpr (SCR) {
          for (int j = 0; j < N; ++j) fS += nt.wsq[j] * fy[j];
          fG = sqrt(frho * fS) / (T * sqrt(T));
        }
        for (int r = fi; r < R; r += FL) {
          const Coef c = coef_of(s_rtab, r);
          double expo =
              c[0] + c[1] * tinv + c[2] * tm13 + c[3] * t13 + c[4] * T + c[5] * t53 + c[6] * lnT;
          double dl = -c[1] * tinv * tinv - (1.0 / 3.0) * c[2] * tm13 * tinv +
                      (1.0 / 3.0) * c[3] * t13 * tinv + c[4] +
                      (5.0 / 3.0) * c[5] * t13 * t13 + c[6] * tinv;
          double hr = 0.0;
          if constexpr (SCR) {
            hr = nt.screen[r];
            expo += hr * fG;
            dl += hr * (-1.5 * fG * tinv);  // d(h G)/dT
          }
          const int4 spv = *reinterpret_cast<const int4 *>(s_rsp + 4 * r);
          const int sp[4] = {spv.x, spv.y, spv.z, spv.w};
          // unconditional slot loads (an absent slot reads entry 0 and
          // stands for 1)
          const double fa = fy[sp[0] < 0 ? 0 : sp[0]];
          const double fb = fy[sp[1] < 0 ? 0 : sp[1]];
          const double fc = fy[sp[2] < 0 ? 0 : sp[2]];
          double pre = exp(expo) * s_emult[r] * c[7];
          // rho^(n_r - 1) for n_r <= 3 reactants
          if (sp[3] >= 2) pre *= frho;
          if (sp[3] >= 3) pre *= frho;
          const double ya = sp[0] >= 0 ? fa : 1.0;
          const double yb = sp[1] >= 0 ? fb : 1.0;
          const double yc = sp[2] >= 0 ? fc : 1.0;
          double full = pre;
          if (sp[0] >= 0) full *= ya;
          if (sp[1] >= 0) full *= yb;
          if (sp[2] >= 0) full *= yc;
          // derivative of the slot product with respect to each slot, and
          // with respect to temperature
          double g[4] = {pre, pre, pre, full * dl};
          if (sp[1] >= 0) g[0] *= yb;
          if (sp[2] >= 0) g[0] *= yc;
          if (sp[0] >= 0) g[1] *= ya;
          if (sp[2] >= 0) g[1] *= yc;
          if (sp[0] >= 0) g[2] *= ya;
          if (sp[1] >= 0) g[2] *= yb;
          const int4 *ro = reinterpret_cast<const int4 *>(s_rout + 8 * r);
          const int4 r0 = ro[0], r1 = ro[1];
          const double qc = s_qcv[r];
#pragma unroll
          for (int aa = 0; aa < 4; ++aa) {
            const int col = (aa < 3) ? sp[aa] : N;
            if (col >= 0) {
              if (!isfinite(g[aa])) jbad = 1;
              const double val = g[aa];
              Unroll<6>::run([&]<int E>() __attribute__((always_inline)) {
                if (E < ne) {
                  const Ent en = ent_of<E>(r0, r1);
                  __hip_atomic_fetch_add(&fM[en.sp * MS + col], en.w * val, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WAVEFRONT);
                }
              });
              __hip_atomic_fetch_add(&fM[N * MS + col], qc * val, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
          }
          if constexpr (SCR) {
            // dR_r/dG = h_r R_r, gathered per row for the rank-one term
            const double u = hr * full;
            Unroll<6>::run([&]<int E>() __attribute__((always_inline)) {
              if (E < ne) {
                const Ent en = ent_of<E>(r0, r1);
                __hip_atomic_fetch_add(&uacc[en.sp], en.w * u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WAVEFRONT);
              }
            });
            __hip_atomic_fetch_add(&uacc[N], qc * u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WAVEFRONT);
          }
        }
      }
      if constexpr (SCR) {
        // rank-one composition term of J: u_i dG/dY_j, dG/dY_j = G A_j^2 / (2 S)
        wave_lds_sync();
        if (fsel >= 0 && asm_j && fi < n) {
          const double ui = uacc[fi] * fG / (2.0 * fS);
          double *mr = fM + fi * MS;
          for (int j = 0; j < N; ++j) mr[j] += ui * nt.wsq[j];
          if (!isfinite(ui)) jbad = 1;
        }
      }
      }  // any_asm
      jbad = gor<FL>(jbad);
      wave_lds_sync();
      if constexpr (!REG_LU) {
        // I - cJ, row by row, from the J just assembled (copied to the
        // cell's area when there is one) or from the one kept there, whose
        // loads go out eight at a time
        if (fsel >= 0 && frow) {
          double *mr = fM + fi * MS;
          const int jo = fsel * MROWS * MROWS + fi;  // the row's first entry in the area
          if (asm_j) {
            for (int j = 0; j < MROWS; ++j) {
              const double v = mr[j];
              if (jw) jw[jo + j * MROWS] = v;
              mr[j] = (fi == j ? 1.0 : 0.0) - fcc * v;
            }
          } else {
            for (int j0 = 0; j0 < MROWS; j0 += 8) {
              double v[8];
#pragma unroll
              for (int u = 0; u < 8; ++u)
                v[u] = j0 + u < MROWS ? jw[jo + (j0 + u) * MROWS] : 0.0;
#pragma unroll
              for (int u = 0; u < 8; ++u)
                if (j0 + u < MROWS) mr[j0 + u] = (fi == j0 + u ? 1.0 : 0.0) - fcc * v[u];
            }
          }
        }
        wave_lds_sync();
      }
      // (c) LU with partial pivoting, one row per lane.  Rows are not moved:
      // `pos` is the position the row would hold after the textbook row swaps
      // (the first largest |pivot| in position order wins).
      int pos = fi;
      int fsing = 0;
      double fdinv = 1.0;
      if constexpr (REG_LU) {
        // The row lives in the lane's LU registers (slot fj is the lane's own
        // cell); per pivot the pivot row's remaining entries go through the
        // y_J area of the slot, which is free once the Jacobian is built.
        const bool mine = fsel >= 0;
        static_assert(!SH::COMPACT, "register factorization keeps all NP rows");
        if (mine) {
          if (asm_j) {
            const double *mr = fM + fi * MS;
#pragma unroll
            for (int j = 0; j < NP; ++j) Jr[j] = mr[j];
            jr_ok = 1;
          }
          // I - cJ
#pragma unroll
          for (int j = 0; j < NP; ++j) LU[0][j] = (fi == j ? 1.0 : 0.0) - fcc * Jr[j];
        }
        wave_lds_sync();
        Unroll<NP>::run([&]<int K>() __attribute__((always_inline)) {
          if (K < n) {
            double v = -2.0;
            int nan_k = 0;
            const bool cand = mine && frow && pos >= K;
            if (cand) {
              v = fabs(LU[0][K]);
              if (v != v) {
                if (pos == K) nan_k = 1;
                v = -1.0;
              }
            }
            int key = cand ? ((pos << 8) | fi) : 0x7fffffff;
            // every row's reciprocal of its entry K, computed while the
            // arg-max runs; the pivot row hands its own over in place of
            // that entry, so no division waits for the pivot row's loads
            const double rown = 1.0 / LU[0][K];
            gargmax_key<FL>(v, key);
            nan_k = gor<FL>(nan_k);
            if (!(v > 0.0) || nan_k) fsing = 1;
            const int bp = key >> 8;
            if (frow) {
              if (pos == K) pos = bp;
              else if (pos == bp) pos = K;
            }
            if (mine && fi == (key & 255)) {
              fy[K] = rown;
#pragma unroll
              for (int j = K + 1; j < NP; ++j) fy[j] = LU[0][j];
            }
            wave_lds_sync();
            // every lane reads its slot's pivot row (in bounds for idle slots
            // too)
            double pr[NP];
#pragma unroll
            for (int j = K; j < NP; ++j) pr[j] = fy[j];
            const double rinv = pr[K];
            if (mine && frow) {
              if (pos == K) fdinv = rinv;
              if (pos > K) {
                const double l = LU[0][K] * rinv;
                LU[0][K] = l;
#pragma unroll
                for (int j = K + 1; j < NP; ++j) LU[0][j] -= l * pr[j];
              }
            }
            wave_lds_sync();
          }
        });
        // rows to LDS in position order, for the hand-over to the solves
        if (mine && frow) {
          double *dst = fM + pos * MS;
#pragma unroll
          for (int j = 0; j < NP; ++j)
            if (!SH::COMPACT || j < n) dst[j] = LU[0][j];
        }
      } else {
        double *Mrow = fM + (frow ? fi : 0) * MS;
        // The pivot at column K: the first largest |entry| in position order
        // among the candidate rows (pos >= K), found by one reduction over
        // the slot's lanes (key: position, then the physical row, the payload;
        // positions of candidates are distinct, so the smallest key is the
        // first position).  Updates pos, fsing and fdinv; returns the pivot's
        // physical row, the row's entry K in mk and the pivot's reciprocal
        // in rk.  With one slot per wave every candidate forms the reciprocal
        // of its entry while the reduction runs and the pivot's is then read
        // from its lane (the pivot is wave-uniform), so no division waits for
        // the pivot to be known; narrower slots divide after the reduction
        // (reading the pivot's lane per slot cost more than it saved).
        auto pivot = [&](int K, double &mk, double &rk) __attribute__((always_inline)) -> int {
          double v = -2.0;
          int nan_k = 0;
          const bool cand = frow && pos >= K;
          mk = 0.0;
          if (cand) {
            mk = Mrow[K];
            v = fabs(mk);
            if (v != v) {
              if (pos == K) nan_k = 1;
              v = -1.0;
            }
          }
          const double rc = FL == 64 ? 1.0 / mk : 0.0;
          int key = cand ? ((pos << 8) | fi) : 0x7fffffff;
          gargmax_key<FL>(v, key);
          if constexpr (FL == 64)
            rk = readlane_f64(rc, __builtin_amdgcn_readfirstlane(key & 63));
          else
            rk = 1.0 / fM[(key & 255) * MS + K];
          const int bp = key >> 8;
          nan_k = gor<FL>(nan_k);
          if (!(v > 0.0) || nan_k) fsing = 1;
          if (frow) {
            if (pos == K) pos = bp;
            else if (pos == bp) pos = K;
          }
          return key & 255;
        };
        // Two columns per pass (the elimination's arithmetic, operation by
        // operation, is the textbook one's): column K's pivot and multipliers
        // l1 and the update of column K + 1 alone; then column K + 1's pivot
        // and multipliers l2, and one sweep over the trailing columns j that
        // applies both updates, a_j - l1 P1_j, then - l2 P2_j with P2 the
        // pivot row of K + 1 after its own column-K update (every lane forms
        // it, P2_j - l1' P1_j with that row's multiplier l1'): the trailing
        // entries are read and written once per two columns.
        for (int K = 0; K < n; K += 2) {
          double mk, rinv1;
          const double *P1 = fM + pivot(K, mk, rinv1) * MS;
          if (frow && pos == K) fdinv = rinv1;
          const bool two = K + 1 < n;
          double l1 = 0.0;
          if (frow && pos > K) {
            l1 = mk * rinv1;
            Mrow[K] = l1;
            if (two) Mrow[K + 1] = fma(-l1, P1[K + 1], Mrow[K + 1]);
          }
          wave_lds_sync();
          if (!two) break;
          double mk2, rinv2;
          const double *P2 = fM + pivot(K + 1, mk2, rinv2) * MS;
          const double l1p = P2[K];  // the multiplier of column K + 1's pivot row at column K
          if (frow && pos == K + 1) fdinv = rinv2;
          const bool below = frow && pos > K + 1;
          double l2 = 0.0;
          if (below) {
            l2 = mk2 * rinv2;
            Mrow[K + 1] = l2;
          }
          if (frow && pos > K) {
            // whole chunks of ECH columns (all loads of a chunk are issued
            // before the first use, so the LDS latency is paid once per
            // chunk), then the remaining columns one by one
            int j0 = K + 2;
            for (; j0 + ECH <= n; j0 += ECH) {
              double a[ECH], b[ECH], c[ECH];
#pragma unroll
              for (int u = 0; u < ECH; ++u) {
                a[u] = Mrow[j0 + u];
                b[u] = P1[j0 + u];
                c[u] = P2[j0 + u];
              }
#pragma unroll
              for (int u = 0; u < ECH; ++u) {
                a[u] = fma(-l1, b[u], a[u]);
                if (below) a[u] = fma(-l2, fma(-l1p, b[u], c[u]), a[u]);
                Mrow[j0 + u] = a[u];
              }
            }
            for (; j0 < n; ++j0) {
              const double b = P1[j0];
              double a = fma(-l1, b, Mrow[j0]);
              if (below) a = fma(-l2, fma(-l1p, b, P2[j0]), a);
              Mrow[j0] = a;
            }
          }
          wave_lds_sync();
        }
      }
      // (d) the factors stay in LDS; publish position -> row and 1/U_pp
      double *aux = fM + (size_t)MROWS * MS;
      if (fsel >= 0) {
        if (frow) {
          aux[pos] = fdinv;
          aux[NP + pos] = (double)fi;
        }
        if (fi == 0) {
          fsc[4 * fj + 2] = (double)fsing;
          fsc[4 * fj + 3] = (double)jbad;
        }
      }
      wave_lds_sync();
      if (myslot >= 0) {
        const double *src = fbase + (size_t)myslot * FB + NP;
        const double *saux = src + (size_t)MROWS * MS;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int p = comp(s);
          if (p < n) {
            // entries j >= n of a row (read inside this slot: the auxiliary
            // rows follow) are replaced by zeros, which the padded columns
            // of the solves' last block of columns multiply
            dinv[s] = saux[p];
            ridx[s] = (int)saux[NP + p];
            // register factorization: rows stored by position
            const double *row = src + (REG_LU ? p : ridx[s]) * MS;
#pragma unroll
            for (int j = 0; j < NP; ++j) LU[s][j] = (!SH::COMPACT || j < n) ? row[j] : 0.0;
          } else {
            dinv[s] = 1.0;
            ridx[s] = p;
#pragma unroll
            for (int j = 0; j < NP; ++j) LU[s][j] = 0.0;
          }
        }
        sing = fsc[4 * myslot + 2] != 0.0;
        if (first_jac && fsc[4 * myslot + 3] != 0.0) {
          // the Jacobian at the initial state is not finite
          status = 3;
          phase = PH_DONE;
          write_state = 0;
        } else {
          cnt[CNT_LU]++;
          lu_ok = 1;
        }
        first_jac = 0;
        // the cell's area now holds J(y_J)
        if constexpr (!REG_LU) jr_ok = jw ? 1 : 0;
      }
      wave_lds_sync();
    }

    double pend = 0.0;
    // a singular Newton matrix is a failed Newton attempt (no RHS needed)
    int nfail = (want && phase == PH_NEWTON && sing) ? 1 : 0;
    if (!defer) fresh_newton = 0;

    // ---------------- C: right-hand side ----------------
    // A cell waiting for its LU already evaluates the first Newton RHS, at
    // the predictor (which the wait does not change), and uses it once the
    // factors are there.
    if (nfail) f_pre = 0;
    const int active = (phase == PH_F0 || phase == PH_F1 || phase == PH_NEWTON) && !nfail;
    const int need_f = active && !f_pre;
    int okf = 1;
    if (need_f) {
      okf = rhs();
      cnt[CNT_RHS]++;
    }
    if (defer) {
      if (need_f) {
        f_pre = 1;
        okf_pre = okf;
      }
    } else if (f_pre) {
      okf = okf_pre;
      f_pre = 0;
    }
    const int do_rhs = active && !defer;  // the right-hand side is used now

    // ---------------- D: what the new right-hand side is used for ----------------
    if (do_rhs) {
      if (phase == PH_F0) {
        if (!okf) {
          status = 3;
          phase = PH_DONE;
        } else {
          // y0 -> D_0, f0 -> D_1 (scaled by h later); initial step size
#pragma unroll
          for (int s = 0; s < S; ++s) {
            Dl[comp(s)] = yv[s];
            Dl[NP + comp(s)] = F[s];
            isc[s] = 1.0 / (atol + rtol * fabs(yv[s]));
          }
          const double d0 = wrms(yv, isc);
          d1 = wrms(F, isc);
          h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
          if (h0 > t_end) h0 = t_end;
          if constexpr (PROBE) probe_h0 = (float)h0;
#pragma unroll
          for (int s = 0; s < S; ++s) yv[s] = yv[s] + h0 * F[s];
          phase = PROBE ? PH_DONE : PH_F1;
        }
      } else if (phase == PH_F1) {
        double df[S];
#pragma unroll
        for (int s = 0; s < S; ++s) df[s] = F[s] - Dl[NP + comp(s)];
        const double d2 = wrms(df, isc) / h0;
        double h1;
        if (!isfinite(d2)) {
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
        h = 100.0 * h0;
        if (h1 < h) h = h1;
        if (t_end < h) h = t_end;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int i = comp(s);
          Dl[NP + i] = h * Dl[NP + i];
#pragma unroll
          for (int j = 2; j < DROWS; ++j) Dl[j * NP + i] = 0.0;
          yJ[s] = Dl[i];
        }
        cnt[CNT_JAC]++;
        jac_cur = 1;
        jr_ok = 0;
        first_jac = 1;
        lu_ok = 0;
        k = 1;
        t = 0.0;
        n_eq = 0;
        need_attempt = 1;
        new_step = 1;
        write_state = 1;
        if constexpr (REC) {
          racc = 1.0;
          if (q == 0) a.sched[cell * a.sched_stride + 1] = h;
        }
        phase = PH_NEWTON;
      } else {  // PH_NEWTON: one modified-Newton iteration
        int fail = !okf;
        int converged = 0;
        if (!fail) {
          double tmp[S];
#pragma unroll
          for (int s = 0; s < S; ++s) tmp[s] = cc * F[s] - psi[s] - dd[s];
          solve(tmp);
          cnt[CNT_SOLVE]++;
          const double dn = wrms(tmp, isc);
          if (!isfinite(dn)) {
            fail = 1;
          } else {
            double rate = 0.0;
            if (it > 0) {
              rate = dn / dprev;
              // predicted error after the remaining iterations,
              // rate^(4 - it) dn / (1 - rate) > tol, with it = 1..3 and
              // 1 - rate > 0 multiplied out
              const double r2 = rate * rate;
              const double rp = it == 1 ? r2 * rate : (it == 2 ? r2 : rate);
              if (rate >= 1.0 || rp * dn > kNewtonTol * (1.0 - rate)) fail = 1;
            }
            if (!fail) {
#pragma unroll
              for (int s = 0; s < S; ++s) {
                yv[s] += tmp[s];
                dd[s] += tmp[s];
              }
              // converged: rate dn / (1 - rate) < tol (here rate < 1)
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
          double e1[S];
          const double rk1 = s_recip[k + 1];
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const double aa = fabs(Dl[comp(s)]), bb = fabs(yv[s]);
            isc[s] = 1.0 / (atol + rtol * (aa > bb ? aa : bb));
            e1[s] = bn_div_by(dd[s], (double)(k + 1), rk1);
          }
          err = wrms(e1, isc);
          if (err > 1.0) {
            double fct = kSafety * exp(bn_log(err) * -rk1);
            if (fct < kMinFactor) fct = kMinFactor;
            h *= fct;
            pend = fct;
            n_eq = 0;
            lu_ok = 0;
            cnt[CNT_REJ]++;
            need_attempt = 1;
          } else {
            // accept: D_{k+2} = d - D_{k+1}, D_{k+1} = d, D_j += D_{j+1}
            t = t_new;
            double em_acc = 0.0, ep_acc = 0.0;
#pragma unroll
            for (int s = 0; s < S; ++s) {
              const int i = comp(s);
              double dr[KMAX + 1];  // rows 0..KMAX, read before the branches on k
#pragma unroll
              for (int j = 0; j <= KMAX; ++j) dr[j] = Dl[j * NP + i];
              const double dk2 = dd[s] - Dl[(k + 1) * NP + i];
              Dl[(k + 1) * NP + i] = dd[s];
              double up = dd[s];
#pragma unroll
              for (int j = KMAX; j >= 0; --j) {
                if (j <= k) {
                  up = dr[j] + up;
                  Dl[j * NP + i] = up;
                }
              }
              if (i < n) {
                const double zm = bn_div_by(Dl[k * NP + i], (double)k, s_recip[k]) * isc[s];
                const double zp = bn_div_by(dk2, (double)(k + 2), s_recip[k + 2]) * isc[s];
                em_acc += zm * zm;
                ep_acc += zp * zp;
              }
            }
            jac_cur = 0;
            n_eq++;
            if constexpr (REC) {
              const int m = cnt[CNT_STEPS];
              if (q == 0 && m < a.sched_cap) {
                double *blk = a.sched + cell * a.sched_stride;
                blk[2 + m] = h;
                blk[2 + a.sched_cap + m] = racc;
                reinterpret_cast<int32_t *>(blk + 2 + 2 * (int64_t)a.sched_cap)[m] = k;
              }
              racc = 1.0;
            }
            cnt[CNT_STEPS]++;
            if (n_eq >= k + 1) {
              em_acc = gsum<L>(em_acc);
              ep_acc = gsum<L>(ep_acc);
              const double em = (k > 1) ? sqrt(bn_div_by(em_acc, dn_sz, inv_n)) : INFINITY;
              const double ep = (k < KMAX) ? sqrt(bn_div_by(ep_acc, dn_sz, inv_n)) : INFINITY;
              // the factors norm^(-1/(order+1)) of orders k-1, k, k+1,
              // compared by their logarithms; one exponential for the best
              const double lm = bn_log(em) * -s_recip[k];
              const double l0 = bn_log(err) * -rk1;
              const double lp = bn_log(ep) * -s_recip[k + 2];
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
              h *= fct;
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
        for (int s = 0; s < S; ++s) {
          yJ[s] = yp[s];
          dd[s] = 0.0;
          yv[s] = yp[s];
        }
        cnt[CNT_JAC]++;
        jac_cur = 1;
        jr_ok = 0;
        lu_ok = 0;
        it = 0;
        fresh_newton = 1;
      } else {
        h *= 0.5;
        n_eq = 0;
        lu_ok = 0;
        need_attempt = 1;
        pend = 0.5;
      }
    }
    if (pend != 0.0 && phase == PH_NEWTON) rescale(k, pend);
  }
  if constexpr (!QUEUE) {
    if constexpr (PROBE) {
      if (phase == PH_DONE && q == 0) a.key[cell] = probe_h0;
    } else {
      if (phase == PH_DONE) write_out();
    }
  }
}

}  // namespace
}  // namespace bn
