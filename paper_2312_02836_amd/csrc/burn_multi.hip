// burn_multi.hip -- the persistent multi-network kernel, its queue-order
// kernels (probe, counting sort, staging), the counter reset kernel, and the
// host-side shape dispatch and LDS sizing for all kernels.
//
// The kernel is built for two waves per SIMD (the narrow shapes, whose
// registers fit half the file) and for one (the wide ones).
//
// Persistent scheduling: the grid is sized to the machine (one or a few
// workgroups per compute unit), not to the work.  Every workgroup walks the
// batch items in the order given (the host puts the costliest cells first);
// for each item it loads the network's tables into LDS once, and its waves
// then take cells from the item's queue counter, one lane group at a time,
// until the counter passes the item's cell count.  A group that finishes a
// cell early takes the next one at once, so cells of uneven stiffness do not
// leave lanes idle until the slowest cell of a static batch is done, and the
// tails of the different networks overlap instead of adding up.
//
// Queue order (ordered launches): a probe runs the burn body of every cell
// up to its initial step size h0, a counting sort over buckets of log2 h0
// ranks the cells stiffest first, and the rank is dealt round-robin into one
// part per XCD.  The cells' arrays are staged in that position order, so a
// workgroup, which takes positions from its own XCD's part first, reads and
// writes lines that the same XCD's L2 holds; the arrays are copied back to
// cell order after the burn.

#include "burn_body.h"

#include <mutex>

#include "burn.h"

namespace bn {

// The workspace of burn_batch_multi_noalloc (queue counters and, for ordered
// launches, the cost-order keys, positions and staged cell arrays).  Every
// device the library runs on holds its own copy until the process ends; the
// calls on one device share it (they must not overlap).  Host code never
// uses this name as an address: noalloc_scratch() looks the device address
// up once per device.
static __device__ __align__(256) unsigned char scratch[BN_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(void **out) {
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_plain_p0(const BurnArgs &a, int L, int S, int block_waves, hipStream_t stream,
                           bool *found);
hipError_t launch_plain_p1(const BurnArgs &a, int L, int S, int block_waves, hipStream_t stream,
                           bool *found);
hipError_t launch_plain_p2(const BurnArgs &a, int L, int S, int block_waves, hipStream_t stream,
                           bool *found);

namespace {

// Shape index sh of the W-waves-per-SIMD set, fixed at compile time.
template <int W, int SH>
__device__ __forceinline__ void run_shape(const BurnArgs &a, const Tabs &tb, double *wb,
                                          unsigned long long *qj) {
  if constexpr (W == 2) {
    if constexpr (SH == 0) run_cells<8, 1, true>(a, tb, wb, 0, qj);
    else if constexpr (SH == 1) run_cells<16, 1, true>(a, tb, wb, 0, qj);
    else if constexpr (SH == 2) run_cells<32, 1, true>(a, tb, wb, 0, qj);
    else run_cells<64, 1, true>(a, tb, wb, 0, qj);
  } else {
    if constexpr (SH == 0) run_cells<4, 4, true>(a, tb, wb, 0, qj);
    else if constexpr (SH == 1) run_cells<16, 2, true>(a, tb, wb, 0, qj);
    else if constexpr (SH == 2) run_cells<32, 1, true>(a, tb, wb, 0, qj);
    else run_cells<64, 1, true>(a, tb, wb, 0, qj);
  }
}

// ONE >= 0: every item has shape ONE (one burn body, the registers of that
// shape alone); ONE < 0: the shape is chosen per item.
template <int W, int ONE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W, W)))
burn_multi_kernel(MultiArgs m) {
  extern __shared__ double smem[];
  __shared__ int s_skip;
  const int wave = threadIdx.x >> 6;
  double *wb = smem + m.tab_doubles + (size_t)wave * m.wave_doubles;
  for (int j = 0; j < m.n_items; ++j) {
    const BurnArgs &a = m.item[j];
    // An item whose queue has already run out is skipped without loading.
    if (threadIdx.x == 0)
      s_skip = __hip_atomic_load(&m.queue[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
               (unsigned long long)a.n_cells;
    __syncthreads();  // every wave is done with the previous item's tables
    const int skip = s_skip;
    if (!skip) load_tables(a.net, a.log_mult, smem);
    __syncthreads();
    if (skip) continue;
    const Tabs tb = tabs_at(smem, a.net.R);
    unsigned long long *qj = m.queue + j;
    if constexpr (ONE >= 0) {
      run_shape<W, ONE>(a, tb, wb, qj);
    } else {
      switch (m.shape[j]) {
        case 0: run_shape<W, 0>(a, tb, wb, qj); break;
        case 1: run_shape<W, 1>(a, tb, wb, qj); break;
        case 2: run_shape<W, 2>(a, tb, wb, qj); break;
        default: run_shape<W, 3>(a, tb, wb, qj); break;
      }
    }
  }
}

// ---- queue order (costliest cells first) ----

// One right-hand side per cell: the integrator's initial step size h0 into
// a.key (static map of cells to lane groups, as the plain kernel).
template <int L, int S>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
burn_probe_kernel(BurnArgs a, int block_waves) {
  using SH = Shape<L, S>;
  extern __shared__ double smem[];
  load_tables(a.net, a.log_mult, smem);
  __syncthreads();
  const Tabs tb = tabs_at(smem, a.net.R);
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  double *wb = smem + tab_doubles_of(a.net.R) + (size_t)wave * SH::wave_doubles(a.net.n);
  const int64_t first = ((int64_t)blockIdx.x * block_waves + wave) * SH::CPW + lane / L;
  run_cells<L, S, false, false, false, false, true>(a, tb, wb, first, nullptr);
}

// Bucket of a cell: two per octave of h0, the smallest steps (the stiffest
// cells, which take the most work) first; +inf and NaN (failed cells) last.
__device__ __forceinline__ int order_bucket(float h0) {
  if (!(h0 < __builtin_inff())) return ORDER_BUCKETS - 1;
  if (!(h0 > 0.0f)) return 0;
  const int b = (int)floorf(2.0f * log2f(h0)) + (ORDER_BUCKETS - 8);
  return b < 0 ? 0 : (b > ORDER_BUCKETS - 1 ? ORDER_BUCKETS - 1 : b);
}

// hist[b] += number of cells in bucket b (per-block counts in LDS first).
__global__ void __launch_bounds__(256) order_hist_kernel(const float *key, int64_t n,
                                                         unsigned *hist) {
  __shared__ unsigned lh[ORDER_BUCKETS];
  for (int b = threadIdx.x; b < ORDER_BUCKETS; b += blockDim.x) lh[b] = 0;
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) atomicAdd(&lh[order_bucket(key[c])], 1u);
  __syncthreads();
  for (int b = threadIdx.x; b < ORDER_BUCKETS; b += blockDim.x)
    if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

// hist[ORDER_BUCKETS + b] = first position of bucket b (exclusive prefix).
__global__ void order_scan_kernel(unsigned *hist) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    unsigned s = 0;
    for (int b = 0; b < ORDER_BUCKETS; ++b) {
      hist[ORDER_BUCKETS + b] = s;
      s += hist[b];
    }
  }
}

// pos[cell] = its queue position: every block reserves a range per bucket,
// then its cells take consecutive positions in it.
__global__ void __launch_bounds__(256) order_scatter_kernel(const float *key, int64_t n,
                                                            unsigned *hist, int32_t *pos) {
  __shared__ unsigned lh[ORDER_BUCKETS], base[ORDER_BUCKETS];
  for (int b = threadIdx.x; b < ORDER_BUCKETS; b += blockDim.x) lh[b] = 0;
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int b = 0;
  unsigned rank = 0;
  if (c < n) {
    b = order_bucket(key[c]);
    rank = atomicAdd(&lh[b], 1u);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < ORDER_BUCKETS; j += blockDim.x)
    base[j] = lh[j] ? atomicAdd(&hist[ORDER_BUCKETS + j], lh[j]) : 0u;
  __syncthreads();
  if (c < n) {
    // cost rank r goes to part r % XCD_PARTS, whose range is contiguous
    const int64_t r = (int64_t)(base[b] + rank);
    const int64_t x = r % XCD_PARTS, per = n / XCD_PARTS, extra = n % XCD_PARTS;
    pos[c] = (int32_t)(x * per + (x < extra ? x : extra) + r / XCD_PARTS);
  }
}

// Staging: position-ordered copies of an item's arrays (one thread per cell,
// reading or writing the caller's arrays in cell order).
__global__ void __launch_bounds__(256) stage_in_kernel(BurnArgs a, BurnArgs st,
                                                       const int32_t *pos) {
  const int64_t n = a.n_cells;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int64_t p = pos[c];
  for (int i = 0; i < a.net.N; ++i) st.Y[(int64_t)i * n + p] = a.Y[(int64_t)i * n + c];
  st.T[p] = a.T[c];
  const_cast<double *>(st.rho)[p] = a.rho[c];
}

__global__ void __launch_bounds__(256) stage_out_kernel(BurnArgs a, BurnArgs st,
                                                        const int32_t *pos) {
  const int64_t n = a.n_cells;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int64_t p = pos[c];
  for (int i = 0; i < a.net.N; ++i) a.Y[(int64_t)i * n + c] = st.Y[(int64_t)i * n + p];
  a.T[c] = st.T[p];
  if (a.status) a.status[c] = st.status[p];
  if (a.counters)
    for (int k = 0; k < 8; ++k) a.counters[(int64_t)k * n + c] = st.counters[(int64_t)k * n + p];
}

__global__ void zero_kernel(unsigned long long *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ULL;
}

template <int L, int S>
size_t wave_doubles_t(int n) {
  return Shape<L, S>::wave_doubles(n);
}

}  // namespace

size_t table_lds_bytes(int R) { return 8 * tab_doubles_of(R); }

size_t wave_lds_bytes(int L, int S, int n) {
#define BN_W(l, s) \
  if (L == l && S == s) return 8 * wave_doubles_t<l, s>(n);
  BN_W(4, 1)
  BN_W(4, 2)
  BN_W(4, 4)
  BN_W(8, 1)
  BN_W(8, 2)
  BN_W(8, 4)
  BN_W(16, 1)
  BN_W(16, 2)
  BN_W(32, 1)
  BN_W(16, 4)
  BN_W(32, 2)
  BN_W(64, 1)
#undef BN_W
  return (size_t)-1;
}

hipError_t launch_plain(const BurnArgs &a, int L, int S, int block_waves, hipStream_t stream) {
  bool found = false;
  hipError_t e = launch_plain_p0(a, L, S, block_waves, stream, &found);
  if (found) return e;
  e = launch_plain_p1(a, L, S, block_waves, stream, &found);
  if (found) return e;
  e = launch_plain_p2(a, L, S, block_waves, stream, &found);
  if (found) return e;
  return hipErrorInvalidValue;
}

hipError_t launch_multi(const MultiArgs &m, int grid, int W, hipStream_t stream) {
  const size_t lds = 8 * (m.tab_doubles + (size_t)m.block_waves * m.wave_doubles);
  const dim3 g((unsigned)grid), blk(64 * m.block_waves);
  int one = m.n_items > 0 ? m.shape[0] : -1;
  for (int j = 1; j < m.n_items; ++j)
    if (m.shape[j] != one) one = -1;
#define BN_MULTI(w, o) hipLaunchKernelGGL((burn_multi_kernel<w, o>), g, blk, lds, stream, m)
  if (W == 2) {
    switch (one) {
      case 0: BN_MULTI(2, 0); break;
      case 1: BN_MULTI(2, 1); break;
      case 2: BN_MULTI(2, 2); break;
      case 3: BN_MULTI(2, 3); break;
      default: BN_MULTI(2, -1); break;
    }
  } else {
    switch (one) {
      case 0: BN_MULTI(1, 0); break;
      case 1: BN_MULTI(1, 1); break;
      case 2: BN_MULTI(1, 2); break;
      case 3: BN_MULTI(1, 3); break;
      default: BN_MULTI(1, -1); break;
    }
  }
#undef BN_MULTI
  return hipGetLastError();
}

template <int L, int S>
hipError_t launch_probe_t(const BurnArgs &a, size_t lds_block, hipStream_t stream) {
  using SH = Shape<L, S>;
  int bw = 4;
  auto lds_of = [&](int w) {
    return 8 * (tab_doubles_of(a.net.R) + (size_t)w * SH::wave_doubles(a.net.n));
  };
  while (bw > 1 && lds_of(bw) > lds_block) bw /= 2;
  if (lds_of(bw) > lds_block) return hipErrorInvalidValue;
  const int64_t cells_per_block = (int64_t)SH::CPW * bw;
  const int64_t blocks = (a.n_cells + cells_per_block - 1) / cells_per_block;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((burn_probe_kernel<L, S>), dim3((unsigned)blocks), dim3(64 * bw), lds_of(bw),
                     stream, a, bw);
  return hipGetLastError();
}

hipError_t launch_order(const BurnArgs &item, float *key, int32_t *pos, unsigned *hist,
                        size_t lds_block, hipStream_t stream) {
  const int64_t n = item.n_cells;
  if (n <= 0) return hipSuccess;
  if (n > 0x7fffffff) return hipErrorInvalidValue;
  BurnArgs a = item;
  a.key = key;
  const int sz = a.net.n;
  hipError_t e = sz <= 8    ? launch_probe_t<8, 1>(a, lds_block, stream)
                 : sz <= 16 ? launch_probe_t<16, 1>(a, lds_block, stream)
                 : sz <= 32 ? launch_probe_t<32, 1>(a, lds_block, stream)
                            : launch_probe_t<64, 1>(a, lds_block, stream);
  if (e != hipSuccess) return e;
  return launch_sort_keys(key, n, pos, hist, stream);
}

hipError_t launch_sort_keys(const float *key, int64_t n, int32_t *pos, unsigned *hist,
                            hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  if (n > 0x7fffffff) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(order_hist_kernel, dim3(blocks), dim3(256), 0, stream, key, n, hist);
  hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(64), 0, stream, hist);
  hipLaunchKernelGGL(order_scatter_kernel, dim3(blocks), dim3(256), 0, stream, key, n, hist, pos);
  return hipGetLastError();
}

hipError_t launch_stage_in(const BurnArgs &a, const BurnArgs &st, const int32_t *pos,
                           hipStream_t stream) {
  if (a.n_cells <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((a.n_cells + 255) / 256);
  hipLaunchKernelGGL(stage_in_kernel, dim3(blocks), dim3(256), 0, stream, a, st, pos);
  return hipGetLastError();
}

hipError_t launch_stage_out(const BurnArgs &a, const BurnArgs &st, const int32_t *pos,
                            hipStream_t stream) {
  if (a.n_cells <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((a.n_cells + 255) / 256);
  hipLaunchKernelGGL(stage_out_kernel, dim3(blocks), dim3(256), 0, stream, a, st, pos);
  return hipGetLastError();
}

hipError_t launch_zero(unsigned long long *p, int n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, stream, p, n);
  return hipGetLastError();
}

}  // namespace bn
