// burn_gen_args.h -- kernel arguments of the generated burn kernels, shared
// by the host code that launches them and the device code compiled at run
// time from a network's generated source.  Plain C types only: the device
// side is compiled without the host headers.
#pragma once

namespace bng {

struct GenArgs {
  double *Y;                      // [N][n_cells] abundances, in/out
  double *T;                      // [n_cells] temperature, in/out
  const double *rho;              // [n_cells]
  int *status;                    // [n_cells] or null
  int *counters;                  // [8][n_cells] or null
  const double *log_mult;         // [R] or null
  double *jws;                    // Jacobian rows of every lane: [entries][n_lanes]
  double *lws;                    // pivoting scratch of every lane: [n*n + 4n][n_lanes]
  unsigned long long *queue;      // the cell counter (unordered launch)
  unsigned long long *parts;      // per-XCD counters (ordered launch) or null
  long long n_cells;
  long long n_lanes;              // grid threads (the workspaces' lane stride)
  double t_end, rtol, atol;
  int max_steps;
  int lu_batch;                   // a factorization pass runs once this many cells want one
  int lu_wait;                    // ... or once a cell has waited this many iterations
  int pad_;
};

}  // namespace bng
