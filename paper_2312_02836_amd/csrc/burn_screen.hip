// burn_screen.hip -- the plain burn of a network whose rates carry the
// synthetic screening factor exp(h_r G(rho, T, Y)) (the paper's network code
// screens its rates, Sec. 2): the factor enters every rate, and the
// Jacobian gets its temperature terms and a rank-one composition part.

#include "burn_body.h"

namespace bn {
namespace {

template <int L, int S, int W>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W, W)))
burn_screen_kernel(BurnArgs a, int block_waves) {
  using SH = Shape<L, S>;
  extern __shared__ double smem[];
  load_tables(a.net, a.log_mult, smem);
  __syncthreads();
  const Tabs tb = tabs_at(smem, a.net.R);
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  double *wb = smem + tab_doubles_of(a.net.R) + (size_t)wave * SH::wave_doubles(a.net.n);
  const int64_t first = ((int64_t)blockIdx.x * block_waves + wave) * SH::CPW + lane / L;
  run_cells<L, S, false, false, false, true>(a, tb, wb, first, nullptr);
}

}  // namespace

hipError_t launch_screen(const BurnArgs &a, int L, int S, int block_waves, hipStream_t stream) {
#define BN_SCR(l, s, w)                                                                          \
  if (L == l && S == s) {                                                                      \
    using SH = Shape<l, s>;                                                                    \
    const size_t lds =                                                                         \
        8 * (tab_doubles_of(a.net.R) + (size_t)block_waves * SH::wave_doubles(a.net.n));       \
    const int64_t per = (int64_t)SH::CPW * block_waves;                                        \
    const int64_t blocks = (a.n_cells + per - 1) / per;                                        \
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;                                      \
    hipLaunchKernelGGL((burn_screen_kernel<l, s, w>), dim3((unsigned)blocks),                  \
                       dim3(64 * block_waves), lds, stream, a, block_waves);                   \
    return hipGetLastError();                                                                  \
  }
  BN_SCR(8, 1, 2)
  BN_SCR(16, 1, 2)
  BN_SCR(32, 1, 2)
  BN_SCR(64, 1, 1)
#undef BN_SCR
  return hipErrorInvalidValue;
}

}  // namespace bn
