// burn_kernels.hip -- FP64 per-cell reaction-network burn for CDNA4 (gfx950).
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
//    row per lane: the Jacobian row is rebuilt from the stored state y_J with
//    static column indices, the LU runs with row-position tracking (no data
//    swaps), and the factors go back to the owning group through LDS.
//  * Control.  Each loop iteration does, per cell: step-attempt setup,
//    the factorization pass (wave-wide), one right-hand side, and the Newton /
//    error-test / step-control logic.  Every heavy routine has one call site,
//    so cells in different phases still share the RHS and solve instructions.

#include "burn_internal.h"

#include <math.h>

namespace bn {
namespace {

constexpr double kSafety = 0.9;
constexpr double kMinFactor = 0.2;
constexpr double kMaxFactor = 10.0;
constexpr double kNewtonTol = 0.03;
constexpr int kNewtonMaxIt = 4;

enum { PH_F0 = 0, PH_F1 = 1, PH_NEWTON = 2, PH_DONE = 3 };
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

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  const long long r = ((long long)(unsigned)lo) | ((long long)hi << 32);
  return __builtin_bit_cast(double, r);
}

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

// broadcast lane SRC (static) of each aligned group of G lanes
template <int G, int SRC>
__device__ __forceinline__ double gbcast(double v) {
  if constexpr (G == 1) {
    return v;
  } else if constexpr (G == 4) {
    return dpp_f64<SRC | (SRC << 2) | (SRC << 4) | (SRC << 6)>(v);
  } else {
    return __shfl(v, SRC, G);
  }
}

// Reduction levels of an aligned group of G lanes.  Each level pairs every
// lane with another (an involution), and after all levels every lane has
// combined all G values: groups of 16/8 use the DPP row mirror / half-row
// mirror, then the quad permutes [2,3,0,1] and [1,0,3,2]; 32/64 use
// ds_bpermute butterflies.
template <int G>
constexpr int n_levels() {
  return G >= 64 ? 6 : G >= 32 ? 5 : G >= 16 ? 4 : G >= 8 ? 3 : G >= 4 ? 2 : G >= 2 ? 1 : 0;
}

template <int G, int LV>
__device__ __forceinline__ double xch(double v) {
  constexpr int NL = n_levels<G>();
  constexpr int FROM_END = NL - 1 - LV;  // 0 = xor 1, 1 = xor 2, 2 = half mirror, 3 = mirror
  if constexpr (G <= 16) {
    if constexpr (FROM_END == 0) return dpp_f64<0xB1>(v);
    else if constexpr (FROM_END == 1) return dpp_f64<0x4E>(v);
    else if constexpr (FROM_END == 2) return dpp_f64<0x141>(v);
    else return dpp_f64<0x140>(v);
  } else {
    return __shfl_xor(v, 1 << FROM_END, G);
  }
}

template <int G, int LV>
__device__ __forceinline__ int xch_i(int v) {
  constexpr int NL = n_levels<G>();
  constexpr int FROM_END = NL - 1 - LV;
  if constexpr (G <= 16) {
    if constexpr (FROM_END == 0) return dpp_i32<0xB1>(v);
    else if constexpr (FROM_END == 1) return dpp_i32<0x4E>(v);
    else if constexpr (FROM_END == 2) return dpp_i32<0x141>(v);
    else return dpp_i32<0x140>(v);
  } else {
    return __shfl_xor(v, 1 << FROM_END, G);
  }
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

template <int G, int LV = 0>
__device__ __forceinline__ int gor(int v) {
  if constexpr (LV < n_levels<G>()) {
    v |= xch_i<G, LV>(v);
    return gor<G, LV + 1>(v);
  } else {
    return v;
  }
}

// Max of v, ties to the smallest p (a total order: all lanes agree).
template <int G, int LV = 0>
__device__ __forceinline__ void gargmax(double &v, int &p) {
  if constexpr (LV < n_levels<G>()) {
    const double ov = xch<G, LV>(v);
    const int op = xch_i<G, LV>(p);
    if (ov > v || (ov == v && op < p)) {
      v = ov;
      p = op;
    }
    gargmax<G, LV + 1>(v, p);
  }
}

// Arg-max with a payload: max of v, ties to the smallest p; w travels with
// the winner.
template <int G, int LV = 0>
__device__ __forceinline__ void gargmax3(double &v, int &p, int &w) {
  if constexpr (LV < n_levels<G>()) {
    const double ov = xch<G, LV>(v);
    const int op = xch_i<G, LV>(p);
    const int ow = xch_i<G, LV>(w);
    if (ov > v || (ov == v && op < p)) {
      v = ov;
      p = op;
      w = ow;
    }
    gargmax3<G, LV + 1>(v, p, w);
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

}  // namespace

// ---------------------------------------------------------------------------
// LDS layout.  Per workgroup (doubles, then ints, then bytes):
//   rtab[R*8] emult[R] q[R] qcv[R] roww[nnz] |
//   rsp[4R] rowoff[N+1] rowr[nnz] coloff[N+1] colent[nsl] | nu8[N*R] | pad
//   rout[8R] (ints)
// Per wave: D[CPW][DS] ybuf[CPW][YS] facc[CPW][YS] fbuf[FC][FB] fsc[FC][4]
// with FB = NP + NP*MS + 2*NP + 1 doubles per factorization slot: y_J (later
// the pivot row), the Newton matrix with row stride MS (later the factors in
// position order) and two auxiliary rows.  The per-cell strides DS and YS are
// 4 doubles more than a multiple of 16 and the matrix row stride MS is odd, so
// the cells of a wave (and the rows of a matrix) fall in different LDS banks.
// ---------------------------------------------------------------------------

struct TabSizes {
  int N, R, nnz, nsl;
  __host__ __device__ size_t doubles() const {
    const size_t d = 8 * (size_t)R + 3 * (size_t)R + nnz;
    const size_t i = 4 * (size_t)R + (N + 1) + nnz + (N + 1) + nsl + 8 * (size_t)R;
    const size_t b = (size_t)N * R;
    return d + (i + 1) / 2 + (b + 7) / 8;
  }
};

template <int L, int S>
struct Shape {
  static constexpr int NP = L * S;
  static constexpr int CPW = 64 / L;
  static constexpr int FL = NP;       // factor lanes per cell (one row each)
  static constexpr int FC = 64 / NP;  // cells per factorization pass
  static_assert(NP == 4 || NP == 8 || NP == 16 || NP == 32 || NP == 64, "NP must be a power of 2");
  static constexpr int DS = DROWS * NP + 4;  // history stride per cell
  static constexpr int YS = NP + 4;          // exchange-vector stride per cell
  static constexpr int MS = NP + 1;          // matrix row stride
  __host__ __device__ static size_t fb(int) { return (size_t)NP * MS + 3 * NP + 1; }
  __host__ __device__ static size_t wave_doubles(int R) {
    return (size_t)CPW * DS + 2 * (size_t)CPW * YS + FC * fb(R) + 4 * FC;
  }
};

template <int L, int S, int W>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W, W)))
burn_plain_kernel(BurnArgs a, int block_waves) {
  using SH = Shape<L, S>;
  constexpr int NP = SH::NP, CPW = SH::CPW, FL = SH::FL, FC = SH::FC;
  constexpr int DS = SH::DS, YS = SH::YS, MS = SH::MS;
  extern __shared__ double smem[];

  const NetTables &nt = a.net;
  const int N = nt.N, R = nt.R, n = nt.n, nnz = nt.nnz, nsl = nt.nsl;
  const TabSizes ts{N, R, nnz, nsl};

  // ---- workgroup tables
  double *s_rtab = smem;
  double *s_emult = s_rtab + 8 * (size_t)R;
  double *s_q = s_emult + R;
  double *s_qcv = s_q + R;
  double *s_roww = s_qcv + R;
  int *s_rsp = reinterpret_cast<int *>(s_roww + nnz);
  int *s_rowoff = s_rsp + 4 * R;
  int *s_rowr = s_rowoff + N + 1;
  int *s_coloff = s_rowr + nnz;
  int *s_colent = s_coloff + N + 1;
  int *s_rout = s_colent + nsl;
  signed char *s_nu = reinterpret_cast<signed char *>(s_rout + 8 * R);
  {
    const int tid = threadIdx.x, nth = blockDim.x;
    for (int i = tid; i < 8 * R; i += nth) s_rtab[i] = nt.rtab[i];
    for (int i = tid; i < R; i += nth) {
      s_emult[i] = a.log_mult ? exp(a.log_mult[i]) : 1.0;
      s_q[i] = nt.q[i];
      s_qcv[i] = nt.q[i] * nt.inv_cv;
    }
    for (int i = tid; i < nnz; i += nth) {
      s_roww[i] = nt.row_w[i];
      s_rowr[i] = nt.row_r[i];
    }
    for (int i = tid; i < 4 * R; i += nth) s_rsp[i] = nt.rsp[i];
    for (int i = tid; i <= N; i += nth) {
      s_rowoff[i] = nt.row_off[i];
      s_coloff[i] = nt.col_off[i];
    }
    for (int i = tid; i < nsl; i += nth) s_colent[i] = nt.col_ent[i];
    for (int i = tid; i < 8 * R; i += nth) s_rout[i] = nt.rout[i];
    for (int i = tid; i < N * R; i += nth) s_nu[i] = nt.nu8[i];
  }
  __syncthreads();

  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int q = lane % L;
  const int cw = lane / L;
  const int64_t C = a.n_cells;
  const int64_t cell = ((int64_t)blockIdx.x * block_waves + wave) * CPW + cw;
  const bool in_range = cell < C;

  double *wb = smem + ts.doubles() + (size_t)wave * SH::wave_doubles(R);
  double *Dl = wb + (size_t)cw * DS;  // this cell's history, [DROWS][NP]
  double *ybuf = wb + (size_t)CPW * DS + (size_t)cw * YS;
  double *facc = wb + (size_t)CPW * DS + (size_t)CPW * YS + (size_t)cw * YS;
  double *fbase = wb + (size_t)CPW * DS + 2 * (size_t)CPW * YS;
  double *fsc = fbase + (size_t)FC * SH::fb(R);

  const double rtol = a.rtol, atol = a.atol, t_end = a.t_end;
  const double rho = in_range ? a.rho[cell] : 1.0;

  // ---- per-lane state (group layout)
  double LU[S][NP];  // factor rows held at positions s*L+q
  double dinv[S];    // 1 / U_pp of those rows
  int ridx[S];       // natural index of those rows
  double yp[S], psi[S], isc[S], dd[S], yv[S], yJ[S], F[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    dinv[s] = 1.0;
    ridx[s] = s * L + q;
#pragma unroll
    for (int j = 0; j < NP; ++j) LU[s][j] = 0.0;
    yp[s] = psi[s] = isc[s] = dd[s] = yv[s] = yJ[s] = F[s] = 0.0;
  }
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
    return sqrt(gsum<L>(acc) / (double)n);
  };

  // change of step size by ratio rh on rows 0..k of D: D <- (R(rh) U)^T D,
  // applied in its two factors (values at the new nodes, then differences)
  auto rescale = [&](int k, double rh) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = comp(s);
      double dcol[KMAX + 1];
#pragma unroll
      for (int b = 0; b <= KMAX; ++b) dcol[b] = (b <= k) ? Dl[b * NP + i] : 0.0;
      double v[KMAX + 1];
#pragma unroll
      for (int m = 0; m <= KMAX; ++m) {
        const double x = (double)m * rh;
        double rb = 1.0;
        double acc = dcol[0];
#pragma unroll
        for (int b = 1; b <= KMAX; ++b) {
          rb *= ((double)(b - 1) - x) * (1.0 / (double)b);
          if (b <= k) acc += rb * dcol[b];
        }
        v[m] = acc;
      }
#pragma unroll
      for (int aa = 0; aa <= KMAX; ++aa) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m <= aa; ++m)
          if (m <= k) acc += u_of(m, aa) * v[m];
        if (aa <= k) Dl[aa * NP + i] = acc;
      }
    }
  };

  // ---- right-hand side F = f(yv) for the own components; 1 if finite.
  // The group's lanes take the reactions r = q, q+L, ...; each rate is added
  // into the accumulator of every species it changes (LDS atomics: lanes of
  // one instruction add in lane order, i.e. in ascending reaction index).
  auto rhs = [&]() __attribute__((always_inline)) -> int {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      ybuf[comp(s)] = yv[s];
      facc[comp(s)] = 0.0;
    }
    wave_lds_sync();
    const double T = ybuf[N];
    const double t13 = cbrt(T);
    const double tm13 = 1.0 / t13;
    const double t53 = T * t13 * t13;
    const double lnT = log(T);
    const double tinv = 1.0 / T;
    double heat = 0.0;
    auto one = [&](int r) __attribute__((always_inline)) {
      const double *c = s_rtab + 8 * (size_t)r;
      const double expo =
          c[0] + c[1] * tinv + c[2] * tm13 + c[3] * t13 + c[4] * T + c[5] * t53 + c[6] * lnT;
      const int *sp = s_rsp + 4 * r;
      double v = exp(expo) * s_emult[r] * c[7];
      for (int i = 1; i < sp[3]; ++i) v *= rho;
      if (sp[0] >= 0) v *= ybuf[sp[0]];
      if (sp[1] >= 0) v *= ybuf[sp[1]];
      if (sp[2] >= 0) v *= ybuf[sp[2]];
      heat += s_q[r] * v;
      const int4 *ro = reinterpret_cast<const int4 *>(s_rout + 8 * r);
      const int4 r0 = ro[0], r1 = ro[1];
      const int ent[7] = {r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
#pragma unroll
      for (int e = 0; e < 6; ++e) {
        if (e < r0.x)
          __hip_atomic_fetch_add(&facc[ent[e] >> 8], (double)(signed char)(ent[e] & 0xff) * v,
                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      }
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
      const double f = (i < N) ? facc[i] : ((i == N) ? heat * nt.inv_cv : 0.0);
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
    for (int s = 0; s < S; ++s) b[s] = ybuf[ridx[s]];
    // forward substitution with the unit lower factor
    Unroll<NP>::run([&]<int K>() __attribute__((always_inline)) {
      if (K < n) {
        const double xk = gbcast<L, K % L>(b[K / L]);
#pragma unroll
        for (int s = K / L; s < S; ++s)
          if (comp(s) > K) b[s] -= LU[s][K] * xk;
      }
    });
    // back substitution with the upper factor
    Unroll<NP>::run([&]<int KK>() __attribute__((always_inline)) {
      constexpr int K = NP - 1 - KK;
      if (K < n) {
        const double xk = gbcast<L, K % L>(b[K / L] * dinv[K / L]);
        if (q == K % L) b[K / L] = xk;
#pragma unroll
        for (int s = 0; s <= K / L; ++s)
          if (comp(s) < K) b[s] -= LU[s][K] * xk;
      }
    });
    wave_lds_sync();
  };

  // ================= cell state machine =================
  int phase = in_range ? PH_F0 : PH_DONE;
  int status = 0, write_state = 0;
  int k = 1, n_eq = 0, jac_cur = 0, lu_ok = 0, it = 0, need_attempt = 0, new_step = 0;
  int fresh_newton = 0, first_jac = 0;
  double t = 0.0, h = 0.0, t_new = 0.0, cc = 0.0, dprev = 0.0, err = 0.0, h0 = 0.0, d1 = 0.0;

  if (in_range) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = comp(s);
      yv[s] = (i < N) ? a.Y[(int64_t)i * C + cell] : ((i == N) ? a.T[cell] : 0.0);
    }
    int bad = !(rho > 0.0) || !isfinite(rho);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = comp(s);
      if (i < n && !isfinite(yv[s])) bad = 1;
      if (i == N && !(yv[s] > 0.0)) bad = 1;
    }
    if (gor<L>(bad)) {
      status = 4;
      phase = PH_DONE;
    }
  }

  while (true) {
    // ---------------- A: start of a step attempt ----------------
    if (phase == PH_NEWTON && need_attempt) {
      if (new_step && cnt[CNT_STEPS] >= a.max_steps) {
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
#pragma unroll
            for (int j = 1; j <= KMAX; ++j) {
              if (j <= k) {
                const double dj = Dl[j * NP + i];
                sa += dj;
                sb += gamma_of(j) * dj;
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
    const int want = (phase == PH_NEWTON && fresh_newton && !lu_ok);
    int sing = 0;
    unsigned long long wmask = __ballot(want && q == 0);
    while (wmask) {
      int sel[FC];
#pragma unroll
      for (int j = 0; j < FC; ++j) {
        if (wmask) {
          sel[j] = (__ffsll((long long)wmask) - 1) / L;
          wmask &= wmask - 1;
        } else {
          sel[j] = -1;
        }
      }
      // (a) the selected cells publish y_J, c and rho
      int myslot = -1;
#pragma unroll
      for (int j = 0; j < FC; ++j)
        if (sel[j] == cw) myslot = j;
      if (myslot >= 0) {
        double *py = fbase + (size_t)myslot * SH::fb(R);
#pragma unroll
        for (int s = 0; s < S; ++s) py[comp(s)] = yJ[s];
        if (q == 0) {
          fsc[4 * myslot + 0] = cc;
          fsc[4 * myslot + 1] = rho;
        }
      }
      wave_lds_sync();
      // (b) factor layout: slot fj = lane / FL, row fi = lane % FL
      const int fj = lane / FL, fi = lane % FL;
      int fsel = -1;
#pragma unroll
      for (int j = 0; j < FC; ++j)
        if (j == fj) fsel = sel[j];
      double *fy = fbase + (size_t)fj * SH::fb(R);
      double *fM = fy + NP;  // Newton matrix [NP][MS], row-major
      const double fcc = fsel >= 0 ? fsc[4 * fj + 0] : 0.0;
      const double frho = fsel >= 0 ? fsc[4 * fj + 1] : 1.0;
#pragma unroll
      for (int j = 0; j < NP; ++j) fM[fi * MS + j] = (fi == j) ? 1.0 : 0.0;
      wave_lds_sync();
      // Rates at y_J for the reactions r = fi, fi+FL, ...; every Jacobian term
      // W(i, r) dR_r/dy_j (W = nu for a species row, q/c_v for the temperature
      // row) is added, times -c, into the Newton matrix I - cJ.
      int jbad = 0;
      if (fsel >= 0) {
        const double T = fy[N];
        const double t13 = cbrt(T);
        const double tm13 = 1.0 / t13;
        const double t53 = T * t13 * t13;
        const double lnT = log(T);
        const double tinv = 1.0 / T;
        for (int r = fi; r < R; r += FL) {
          const double *c = s_rtab + 8 * (size_t)r;
          const double expo =
              c[0] + c[1] * tinv + c[2] * tm13 + c[3] * t13 + c[4] * T + c[5] * t53 + c[6] * lnT;
          const double dl = -c[1] * tinv * tinv - (1.0 / 3.0) * c[2] * tm13 * tinv +
                            (1.0 / 3.0) * c[3] * t13 * tinv + c[4] +
                            (5.0 / 3.0) * c[5] * t13 * t13 + c[6] * tinv;
          const int *sp = s_rsp + 4 * r;
          double pre = exp(expo) * s_emult[r] * c[7];
          for (int i = 1; i < sp[3]; ++i) pre *= frho;
          const double ya = sp[0] >= 0 ? fy[sp[0]] : 1.0;
          const double yb = sp[1] >= 0 ? fy[sp[1]] : 1.0;
          const double yc = sp[2] >= 0 ? fy[sp[2]] : 1.0;
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
          const int ent[7] = {r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
          const double qc = s_qcv[r];
#pragma unroll
          for (int aa = 0; aa < 4; ++aa) {
            const int col = (aa < 3) ? sp[aa] : N;
            if (col >= 0) {
              if (!isfinite(g[aa])) jbad = 1;
              const double val = -fcc * g[aa];
#pragma unroll
              for (int e = 0; e < 6; ++e) {
                if (e < r0.x)
                  __hip_atomic_fetch_add(&fM[(ent[e] >> 8) * MS + col],
                                         (double)(signed char)(ent[e] & 0xff) * val,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
              }
              __hip_atomic_fetch_add(&fM[N * MS + col], qc * val, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
          }
        }
      }
      jbad = gor<FL>(jbad);
      wave_lds_sync();
      // (c) LU with partial pivoting on the matrix in LDS, one row per lane.
      // Rows are not moved: `pos` is the position the row would hold after the
      // textbook row swaps (the first largest |pivot| in position order wins).
      int pos = fi;
      int fsing = 0;
      double fdinv = 1.0;
      double *Mrow = fM + fi * MS;
      for (int K = 0; K < n; ++K) {
        double v = -2.0;
        int nan_k = 0;
        if (pos >= K) {
          v = fabs(Mrow[K]);
          if (v != v) {
            if (pos == K) nan_k = 1;
            v = -1.0;
          }
        }
        int bp = (pos >= K) ? pos : (1 << 30);
        int prow_i = fi;  // physical row of the pivot (payload of the arg-max)
        gargmax3<FL>(v, bp, prow_i);
        nan_k = gor<FL>(nan_k);
        if (!(v > 0.0) || nan_k) fsing = 1;
        if (pos == K) pos = bp;
        else if (pos == bp) pos = K;
        const double *P = fM + prow_i * MS;
        const double rinv = 1.0 / P[K];
        if (pos == K) fdinv = rinv;
        if (pos > K) {
          const double l = Mrow[K] * rinv;
          Mrow[K] = l;
          for (int j = K + 1; j < n; ++j) Mrow[j] -= l * P[j];
        }
        wave_lds_sync();
      }
      // (d) the factors stay in LDS; publish position -> row and 1/U_pp
      double *aux = fM + NP * MS;
      if (fsel >= 0) {
        aux[pos] = fdinv;
        aux[NP + pos] = (double)fi;
        if (fi == 0) {
          fsc[4 * fj + 2] = (double)fsing;
          fsc[4 * fj + 3] = (double)jbad;
        }
      }
      wave_lds_sync();
      if (myslot >= 0) {
        const double *src = fbase + (size_t)myslot * SH::fb(R) + NP;
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int p = comp(s);
          dinv[s] = src[NP * MS + p];
          ridx[s] = (int)src[NP * MS + NP + p];
          const double *row = src + ridx[s] * MS;
#pragma unroll
          for (int j = 0; j < NP; ++j) LU[s][j] = row[j];
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
      }
      wave_lds_sync();
    }

    double pend = 0.0;
    // a singular Newton matrix is a failed Newton attempt (no RHS needed)
    int nfail = (want && phase == PH_NEWTON && sing) ? 1 : 0;
    fresh_newton = 0;

    // ---------------- C: right-hand side ----------------
    const int do_rhs = (phase != PH_DONE) && !nfail;
    int okf = 1;
    if (do_rhs) {
      okf = rhs();
      cnt[CNT_RHS]++;
    }

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
#pragma unroll
          for (int s = 0; s < S; ++s) yv[s] = yv[s] + h0 * F[s];
          phase = PH_F1;
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
              double rp = rate;  // rate^(4 - it)
              for (int e = it + 1; e < kNewtonMaxIt; ++e) rp *= rate;
              if (rate >= 1.0 || rp / (1.0 - rate) * dn > kNewtonTol) fail = 1;
            }
            if (!fail) {
#pragma unroll
              for (int s = 0; s < S; ++s) {
                yv[s] += tmp[s];
                dd[s] += tmp[s];
              }
              if (dn == 0.0 || (it > 0 && rate / (1.0 - rate) * dn < kNewtonTol)) {
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
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const double aa = fabs(Dl[comp(s)]), bb = fabs(yv[s]);
            isc[s] = 1.0 / (atol + rtol * (aa > bb ? aa : bb));
            e1[s] = dd[s] / (double)(k + 1);
          }
          err = wrms(e1, isc);
          if (err > 1.0) {
            double fct = kSafety * pow(err, -1.0 / (double)(k + 1));
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
              const double dk2 = dd[s] - Dl[(k + 1) * NP + i];
              Dl[(k + 1) * NP + i] = dd[s];
              double up = dd[s];
              for (int j = k; j >= 0; --j) {
                up = Dl[j * NP + i] + up;
                Dl[j * NP + i] = up;
              }
              if (i < n) {
                const double zm = (Dl[k * NP + i] / (double)k) * isc[s];
                const double zp = (dk2 / (double)(k + 2)) * isc[s];
                em_acc += zm * zm;
                ep_acc += zp * zp;
              }
            }
            jac_cur = 0;
            n_eq++;
            cnt[CNT_STEPS]++;
            if (n_eq >= k + 1) {
              em_acc = gsum<L>(em_acc);
              ep_acc = gsum<L>(ep_acc);
              const double em = (k > 1) ? sqrt(em_acc / (double)n) : INFINITY;
              const double ep = (k < KMAX) ? sqrt(ep_acc / (double)n) : INFINITY;
              const double fm = pow(em, -1.0 / (double)k);
              const double f0 = pow(err, -1.0 / (double)(k + 1));
              const double fp = pow(ep, -1.0 / (double)(k + 2));
              double best = f0;
              int dk = 0;
              if (fm > best) {
                best = fm;
                dk = -1;
              }
              if (fp > best) {
                best = fp;
                dk = 1;
              }
              k += dk;
              double fct = kSafety * best;
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

    if (__ballot(phase != PH_DONE) == 0) break;
  }
  if (write_state) cnt[CNT_ORDER] = k;

  // ---- outputs
  if (in_range) {
    if (write_state) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int i = comp(s);
        if (i < N) a.Y[(int64_t)i * C + cell] = Dl[i];
        else if (i == N) a.T[cell] = Dl[i];
      }
    }
    if (q == 0) {
      if (a.status) a.status[cell] = status;
      if (a.counters) {
#pragma unroll
        for (int c = 0; c < 8; ++c) a.counters[(int64_t)c * C + cell] = (status == 4) ? 0 : cnt[c];
      }
    }
  }
}

// ---------------------------------------------------------------------------

bool choose_shape(int n, int lanes_hint, int *L, int *S) {
  struct Sh {
    int L, S;
  };
  static const Sh shapes[] = {{4, 1}, {4, 2}, {4, 4}, {8, 4}, {16, 4}};
  for (const Sh &sh : shapes) {
    if (lanes_hint && sh.L != lanes_hint) continue;
    if (sh.L * sh.S >= n) {
      *L = sh.L;
      *S = sh.S;
      return true;
    }
  }
  return false;
}

template <int L, int S>
static size_t lds_bytes_t(const BurnArgs &a, int block_waves) {
  const TabSizes ts{a.net.N, a.net.R, a.net.nnz, a.net.nsl};
  return 8 * (ts.doubles() + (size_t)block_waves * Shape<L, S>::wave_doubles(a.net.R));
}

template <int L, int S, int W>
static hipError_t launch_one(const BurnArgs &a, int block_waves, hipStream_t stream) {
  constexpr int CPW = 64 / L;
  const size_t lds = lds_bytes_t<L, S>(a, block_waves);
  const int64_t cells_per_block = (int64_t)CPW * block_waves;
  const int64_t blocks = (a.n_cells + cells_per_block - 1) / cells_per_block;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((burn_plain_kernel<L, S, W>), dim3((unsigned)blocks), dim3(64 * block_waves),
                     lds, stream, a, block_waves);
  return hipGetLastError();
}

size_t plain_lds_bytes(const BurnArgs &a, int L, int S, int block_waves) {
#define BN_CASE(l, s) \
  if (L == l && S == s) return lds_bytes_t<l, s>(a, block_waves);
  BN_CASE(4, 1)
  BN_CASE(4, 2)
  BN_CASE(4, 4)
  BN_CASE(8, 4)
  BN_CASE(16, 4)
#undef BN_CASE
  return (size_t)-1;
}

hipError_t launch_plain(const BurnArgs &a, int L, int S, int block_waves, hipStream_t stream) {
#define BN_CASE(l, s, w) \
  if (L == l && S == s) return launch_one<l, s, w>(a, block_waves, stream);
  BN_CASE(4, 1, 2)
  BN_CASE(4, 2, 2)
  BN_CASE(4, 4, 1)
  BN_CASE(8, 4, 1)
  BN_CASE(16, 4, 1)
#undef BN_CASE
  return hipErrorInvalidValue;
}

}  // namespace bn
