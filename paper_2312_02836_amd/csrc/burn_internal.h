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
  const int *rout;     // [R][8]: count, then (species << 8) | (nu_ir & 0xff) for nu_ir != 0
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
};

// Kernel variants: lanes per cell L and slots per lane S (system padded to
// L*S components).  Returns hipSuccess or the launch error.
hipError_t launch_plain(const BurnArgs &a, int L, int S, int block_waves, hipStream_t stream);

// Choose (L, S) for a system of size n; returns false if unsupported.
bool choose_shape(int n, int lanes_hint, int *L, int *S);

}  // namespace bn
