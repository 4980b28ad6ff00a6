// burn_plain.h -- the plain kernel: one launch per network, cells mapped
// statically to lane groups (cell = (workgroup * waves + wave) * cells per
// wave + group).  Each burn_plain_p*.hip instantiates a few shapes, so the
// shapes compile in parallel.
#pragma once

#include "burn_body.h"

namespace bn {
namespace {

template <int L, int S, int W>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W, W)))
burn_plain_kernel(BurnArgs a, int block_waves) {
  using SH = Shape<L, S>;
  extern __shared__ double smem[];
  load_tables(a.net, a.log_mult, smem);
  __syncthreads();
  const Tabs tb = tabs_at(smem, a.net.R);
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  double *wb = smem + tab_doubles_of(a.net.R) + (size_t)wave * SH::wave_doubles(a.net.n);
  const int64_t first = ((int64_t)blockIdx.x * block_waves + wave) * SH::CPW + lane / L;
  run_cells<L, S, false>(a, tb, wb, first, nullptr);
}

template <int L, int S, int W>
hipError_t launch_plain_t(const BurnArgs &a, int block_waves, hipStream_t stream) {
  using SH = Shape<L, S>;
  const size_t lds = 8 * (tab_doubles_of(a.net.R) + (size_t)block_waves * SH::wave_doubles(a.net.n));
  const int64_t cells_per_block = (int64_t)SH::CPW * block_waves;
  const int64_t blocks = (a.n_cells + cells_per_block - 1) / cells_per_block;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((burn_plain_kernel<L, S, W>), dim3((unsigned)blocks), dim3(64 * block_waves),
                     lds, stream, a, block_waves);
  return hipGetLastError();
}

}  // namespace
}  // namespace bn

#define BN_PLAIN_CASE(l, s, w) \
  if (L == l && S == s) {      \
    *found = true;             \
    return launch_plain_t<l, s, w>(a, block_waves, stream); \
  }
