// Internal interface between the C ABI (burn_api.cpp) and the kernels
// (burn_kernels.hip).  Not installed; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bn {

constexpr int KMAX = 5;           // highest BDF order
constexpr int DROWS = KMAX + 2;   // stored backward differences D_0..D_{k+1}
constexpr int RTAB = 8;           // doubles per reaction in the rate table: a0..a6, 1/prod(m!)

// Device copies of a network's tables (owned by a bn_network).
struct NetTables {
  int N;          // species
  int R;          // reactions
  int n;          // system size N + 1 (temperature last)
  int nnz;        // entries of the species-row stoichiometry lists
  double inv_cv;  // 1 / c_v
  const double *rtab;  // [R][RTAB]
  const double *q;     // [R] heat per event
  const int *rsp;      // [R][4] reactant species per slot (-1 = empty), then n_r
  const int *row_off;  // [N + 1] start of each species' list in row_r / row_w
  const int *row_r;    // [nnz] reaction index (ascending within a species)
  const double *row_w; // [nnz] net stoichiometric coefficient nu_ir (nonzero)
  int nsl;             // used reactant slots over all reactions
  const int *col_off;  // [N + 1] start of each species' reactant-slot list
  const int *col_ent;  // [nsl] (r << 2) | slot, ascending in r then slot
  const signed char *nu8;  // [N][R] dense nu_ir
  const int *rout;     // [R][8]: count, then (species << 8) | (nu_ir & 0xff) for nu_ir != 0,
                       // padded to 6 entries with coefficient 0 on the first species
  int max_ent;         // largest count in rout (0..6)
  const double *screen;  // [R] screening strengths h_r, or nullptr
  const double *wsq;     // [N] A_j^2 (screening)
};

struct BurnArgs {
  NetTables net;
  int64_t n_cells;
  double *Y;          // [N][n_cells]
  const double *rho;  // [n_cells]
  double *T;          // [n_cells]
  const double *log_mult;  // [R] or nullptr
  int32_t *status;    // [n_cells] or nullptr
  int32_t *counters;  // [8][n_cells] or nullptr
  double t_end, rtol, atol;
  int max_steps;
  // Schedule recording (sensitivity runs; nullptr otherwise): per cell a
  // block of sched_stride doubles at sched + cell * sched_stride holding
  // [0] accepted steps (-1 if the cell failed), [1] initial step size,
  // [2, 2 + cap) step sizes, [2 + cap, 2 + 2 cap) rescale ratios, then cap
  // int32 orders.
  double *sched;
  int64_t sched_stride;
  int sched_cap;
  // Constant per-cell source [n][n_cells] added to the right-hand side
  // (simplified-SDC forcing; nullptr otherwise).
  const double *src;
  // Order probe: per cell the integrator's initial step size h0
  // (+inf for a cell that fails before it), [n_cells].
  float *key;
  // Persistent kernel, ordered launch: XCD_PARTS zeroed queue counters.
  // Positions are split into XCD_PARTS interleaved parts (part x holds the
  // x-th, (x+8)-th, ... cells of the cost order, as one contiguous range);
  // a workgroup takes positions from the part of its XCD and, when that is
  // exhausted, from the others.  nullptr: one counter (MultiArgs::queue).
  unsigned long long *parts;
  // Shapes that factor in LDS (not in registers): per wave of the launch
  // grid an area of jws_wave doubles, one rows x rows block per cell of the
  // wave (column-major), that keeps the cell's J(y_J) from its assembly
  // until the Jacobian is refreshed; the passes between form I - cJ from it
  // instead of assembling J again.  nullptr: every pass assembles J.
  double *jws;
  int64_t jws_wave;
};
constexpr int XCD_PARTS = 8;  // MI355X: workgroup b runs on XCD b % 8

// Shapes: lanes per cell L, slots per lane S (the system is padded to
// NP = L*S components) and the waves per SIMD W the kernel is compiled for
// (W = 2 for the shapes whose registers fit half the file).  Plain kernels
// exist for every PLAIN_SHAPES entry.  The persistent kernel is built twice:
// for W = 2 with the shapes of MULTI_SHAPES_2 and for W = 1 with those of
// MULTI_SHAPES_1; the recording, source and screened kernels use
// MULTI_SHAPES_2 (with (64,1) at W = 1).
struct ShapeLS {
  int L, S, W;
};
constexpr ShapeLS PLAIN_SHAPES[] = {{4, 1, 2},  {4, 2, 2},  {4, 4, 1},  {8, 1, 2},
                                    {8, 2, 2},  {8, 4, 1},  {16, 1, 2}, {16, 2, 1},
                                    {32, 1, 2}, {16, 4, 1}, {32, 2, 1}, {64, 1, 1}};
constexpr int N_PLAIN_SHAPES = 12;
constexpr ShapeLS MULTI_SHAPES_2[] = {{8, 1, 2}, {16, 1, 2}, {32, 1, 2}, {64, 1, 2}};
constexpr ShapeLS MULTI_SHAPES_1[] = {{4, 4, 1}, {16, 2, 1}, {32, 1, 1}, {64, 1, 1}};
constexpr int N_MULTI_SHAPES = 4;

// LDS bytes of the network tables and of one wave's working area.
size_t table_lds_bytes(int R);
size_t wave_lds_bytes(int L, int S, int n);

// One launch of the plain kernel: cells map statically to lane groups.
hipError_t launch_plain(const BurnArgs &a, int L, int S, int block_waves, hipStream_t stream);

// The persistent multi-network launch: every workgroup walks the items in
// order, and its waves take cells of the current item from that item's
// device queue counter until it passes n_cells.
constexpr int MAX_ITEMS = 8;
struct MultiArgs {
  BurnArgs item[MAX_ITEMS];
  int shape[MAX_ITEMS];           // index into MULTI_SHAPES_2 or MULTI_SHAPES_1
  unsigned long long *queue;      // [n_items] counters, zeroed before the launch
  int n_items;
  int block_waves;
  size_t tab_doubles;             // LDS doubles reserved for tables (max over items)
  size_t wave_doubles;            // LDS doubles per wave area (max over items)
};
hipError_t launch_multi(const MultiArgs &m, int grid, int W, hipStream_t stream);

// Device address of the current device's copy of the static scratch array
// (BN_NOALLOC_SCRATCH_BYTES bytes, 256-byte aligned) that
// burn_batch_multi_noalloc uses as its workspace; looked up once per device.
hipError_t noalloc_scratch(void **out);

// Queue order of one item of the persistent kernel, costliest cells first:
// a probe launch computes every cell's initial step size h0 (one right-hand
// side), then a counting sort over ORDER_BUCKETS buckets of log2 h0 gives
// every cell its position pos[cell].  hist is 2 * ORDER_BUCKETS
// zero-initialized counters.  The item's arrays are then staged in position
// order (stage_in), burnt in index order, and written back (stage_out), so
// that cells that run at nearby times also share memory lines.
constexpr int ORDER_BUCKETS = 128;
hipError_t launch_order(const BurnArgs &a, float *key, int32_t *pos, unsigned *hist,
                        size_t lds_block, hipStream_t stream);
// The counting sort alone: pos[c] for n keys (smallest first, 128 buckets of
// two per octave, positions dealt into XCD_PARTS parts as for the queue).
hipError_t launch_sort_keys(const float *key, int64_t n, int32_t *pos, unsigned *hist,
                            hipStream_t stream);
// staged copy of an item: st.Y, st.T, st.rho, st.status, st.counters point
// to position-ordered arrays of the item's size (status/counters null when
// the item's are)
hipError_t launch_stage_in(const BurnArgs &a, const BurnArgs &st, const int32_t *pos,
                           hipStream_t stream);
hipError_t launch_stage_out(const BurnArgs &a, const BurnArgs &st, const int32_t *pos,
                            hipStream_t stream);

// Sensitivity runs (discrete adjoint with respect to the log-rate
// multipliers).  The replay / adjoint kernels take one cell per 32 lanes for
// systems of up to 32 components, else one per wave.
struct AdjArgs {
  NetTables net;
  int64_t n_cells;
  const double *Y0, *rho, *T0, *log_mult;
  double *Yout, *Tout, *Eout;  // replayed end state and released energy (forward)
  const double *gY, *gE;        // cotangents (backward)
  double *grad;                 // [R][n_cells] (backward)
  int32_t *status;              // [n_cells] (forward: read and updated; backward: read)
  int32_t *iters;               // [2][n_cells] or nullptr: replay Newton iterations and
                                // factorizations (forward)
  double *sched;                // schedule blocks (see BurnArgs)
  int64_t sched_stride;
  int sched_cap;
  double *ckpt;                 // [n_cells][n_ckpt][7][n]
  int n_ckpt;
  double *seg;                  // [n_cells][adjoint_seg_doubles(n)]: corrected states of
                                // the segment being reversed (backward)
  const int32_t *order;         // [n_cells] cell at each position (costliest first), or
                                // nullptr for index order
  double *states;               // pool of corrected states (forward writes, backward reads)
  int64_t *soff;                // [n_cells] a cell's first state in the pool (doubles), or
                                // -1 when its states do not fit (it keeps the recompute path)
  int64_t states_cap;           // doubles in the pool
  double rtol, atol;
  int part;                     // backward: 0 every cell, 1 the cells whose states are in
                                // the pool, 2 the others (set by launch_adjoint)
};
size_t adjoint_sched_stride(int cap);  // doubles per cell
int adjoint_n_ckpt(int cap);
size_t adjoint_seg_doubles(int n);    // per cell
size_t adjoint_lds_bytes(int R, int n, int waves);
int adjoint_cells_per_wave(int n);
// The recording run on a persistent grid of `grid` workgroups taking cells
// from *queue (one zeroed counter).
hipError_t launch_record_queue(const BurnArgs &a, int L, int S, int block_waves, int grid,
                               unsigned long long *queue, hipStream_t stream);
// Order of the cells for the replay and reverse sweep, from the recorded
// step counts (most steps first): key, pos and hist are scratch (hist zeroed
// by the call), order receives the cell at each position.
hipError_t launch_adjoint_order(const AdjArgs &a, float *key, int32_t *pos, unsigned *hist,
                                int32_t *order, hipStream_t stream);
// Places the cells' corrected states in the pool: from the recorded step
// counts (a single workgroup scan, cells in index order), soff[c] = the
// offset of cell c's n * steps doubles, or -1 for a cell whose states do not
// fit in a.states_cap or whose recording failed.
hipError_t launch_adjoint_states(const AdjArgs &a, hipStream_t stream);
// simd_waves: 3 or 2, the register budget of the kernel instance to launch
hipError_t launch_adjoint(const AdjArgs &a, bool backward, int waves, int simd_waves,
                          hipStream_t stream);

// Plain launch with a constant per-cell source (a.src != nullptr); shapes
// of MULTI_SHAPES_2.
hipError_t launch_source(const BurnArgs &a, int L, int S, int block_waves, hipStream_t stream);

// Plain launch of a screened network (a.net.screen != nullptr); shapes of
// MULTI_SHAPES_2.
hipError_t launch_screen(const BurnArgs &a, int L, int S, int block_waves, hipStream_t stream);

// Zero n counters with a kernel (no memset node, so the sequence can be
// captured into a graph and replayed).
hipError_t launch_zero(unsigned long long *p, int n, hipStream_t stream);

}  // namespace bn
