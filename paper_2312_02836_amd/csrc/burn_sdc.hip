// burn_sdc.hip -- the plain burn with a constant per-cell source added to the
// right-hand side, dy/dt = f(y) + A_adv: the form in which a simplified-SDC
// coupling hands a zone's advective change to the reaction integration (the
// network code couples to the hydrodynamics that way, paper Sec. 2).  The
// source does not enter the Jacobian.

#include "burn_body.h"

namespace bn {
namespace {

template <int L, int S, int W>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W, W)))
burn_source_kernel(BurnArgs a, int block_waves) {
  using SH = Shape<L, S>;
  extern __shared__ double smem[];
  load_tables(a.net, a.log_mult, smem);
  __syncthreads();
  const Tabs tb = tabs_at(smem, a.net.R);
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  double *wb = smem + tab_doubles_of(a.net.R) + (size_t)wave * SH::wave_doubles(a.net.n);
  const int64_t first = ((int64_t)blockIdx.x * block_waves + wave) * SH::CPW + lane / L;
  run_cells<L, S, false, false, true>(a, tb, wb, first, nullptr);
}

}  // namespace

hipError_t launch_source(const BurnArgs &a, int L, int S, int block_waves, hipStream_t stream) {
#define BN_SRC(l, s, w)                                                                          \
  if (L == l && S == s) {                                                                      \
    using SH = Shape<l, s>;                                                                    \
    const size_t lds =                                                                         \
        8 * (tab_doubles_of(a.net.R) + (size_t)block_waves * SH::wave_doubles(a.net.n));       \
    const int64_t per = (int64_t)SH::CPW * block_waves;                                        \
    const int64_t blocks = (a.n_cells + per - 1) / per;                                        \
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;                                      \
    hipLaunchKernelGGL((burn_source_kernel<l, s, w>), dim3((unsigned)blocks),                  \
                       dim3(64 * block_waves), lds, stream, a, block_waves);                   \
    return hipGetLastError();                                                                  \
  }
  BN_SRC(8, 1, 2)
  BN_SRC(16, 1, 2)
  BN_SRC(32, 1, 2)
  BN_SRC(64, 1, 1)
#undef BN_SRC
  return hipErrorInvalidValue;
}

}  // namespace bn
